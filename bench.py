#!/usr/bin/env python3
"""Throughput of the adaptive-velocity-space sweep on one MI355X.

Workload: 2-D Ma 5 flow past a cylinder (the shape of the paper's Sec. 4.1
case): body-fitted O-grid 128 (r) x 256 (theta), outer radius 15 D, quadtree
velocity mesh on [-15, 15]^2 with 32^2 roots and 3 levels, C1 calibrated so
that the step-0 tree holds about ``--leaves`` leaves.  Synthetic seeded
bow-shock state (no flow data is available).

One timed step = one adaptation cycle of the hot path: ``--nu`` explicit
sweeps (reconstruction, interface flux, moments, conservative Shakhov
relaxation), then the criterion, the new tree and remap plan, and the
consanguinity remap with its conservation correction.  ``value`` counts
cells x leaves x sweeps per second of that whole cycle, inputs resident in
HBM.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell×velocity-node updates/s, FP64 plain vs FP32/batched form; % HBM roofline"
HBM_PEAK = 8.0e12
VALU_PEAK = 78.6e12      # FP vector, FP64 or unpacked FP32: 256 CU x 64 lanes x 2 flop x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--nu", type=int, default=20, help="sweeps per adaptation cycle")
    p.add_argument("--leaves", type=int, default=20000, help="target leaf count of the step-0 tree")
    p.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    p.add_argument("--forms", action="store_true", help="also time the FP32 form and the batched form")
    p.add_argument("--ncase", type=int, default=64, help="cases of the batched form")
    p.add_argument("--train-events", type=int, default=24, help="adaptation events labelled for the learned form")
    p.add_argument("--train-rows", type=int, default=1_200_000, help="label capacity of the learned form")
    p.add_argument("--train-epochs", type=int, default=4)
    p.add_argument("--sphere-C1", type=float, default=1.0076e-4, help="splitting threshold of the 3-D form (~20k leaves)")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--one-form", action="store_true", help="time only --precision (not also the other precision)")
    p.add_argument("--no-sweep", action="store_true", help="skip the extra sweep-only timing (profiling runs)")
    p.add_argument("--no-batched", action="store_true", help="skip the batched form (profiling runs)")
    p.add_argument("--only", choices=["sphere", "learned", "batched"],
                   help="run only this form and print its record (profiling runs; not the benchmark line)")
    p.add_argument("--copy-probe", type=float, default=0.0,
                   help="GiB copied device-to-device by torch before the run (calibrates HBM byte counters)")
    p.add_argument("--nr", type=int, default=128)
    p.add_argument("--nth", type=int, default=256)
    # C1 for a ~2e4-leaf step-0 tree on this workload, found once by the --calibrate bisection
    p.add_argument("--C1", type=float, default=1.74658e-06, help="splitting threshold (C2 = e^-8 C1)")
    p.add_argument("--calibrate", action="store_true", help="bisect C1 for --leaves instead of using --C1")
    return p.parse_args()


class Workload:
    def __init__(self, args, precision):
        import torch
        from paper_2212_05645_amd import avs
        from workloads import fields as F
        self.torch, self.avs = torch, avs
        self.cfg = F.cylinder(nr=args.nr, nth=args.nth)
        c = self.cfg
        cap = 32 * 32 * 64
        self.cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], c['venkat_K'], c['prim0'],
                           precision=avs.AVS_FP32 if precision == "fp32" else avs.AVS_FP64, leaf_capacity=cap)
        L = self.cs.leaves()
        self.base_level, self.base_idx = L['level'].copy(), L['idx'].copy()
        self.W0 = self.cs.get_W()
        self.nc = self.cs.nc
        self.nf = int(c['mesh']['nfaces'])

    def tree(self, C1):
        """Step-0 tree: roots, then one adaptation per level on cells and probes."""
        cs, c = self.cs, self.cfg
        cs.set_leaves(self.base_level, self.base_idx)
        cs.set_state(None, self.W0)
        for _ in range(c['vspace']['max_level']):
            try:
                cs.adapt(C1, math.exp(-8.0) * C1, probes=c['probes'])
            except self.avs.AvsError as e:
                if e.status == self.avs.AVS_E_CAPACITY:
                    return None
                raise
            cs.remap(2)
        cs.set_state(None, self.W0)
        return cs.nleaves()

    def calibrate(self, target):
        lo, hi = -8.0, -1.0
        best = None
        for it in range(16):
            mid = 0.5 * (lo + hi)
            n = self.tree(10.0 ** mid)
            log(f"calibrate: C1=1e{mid:.4f} -> {n} leaves")
            if n is None or n > target:
                lo = mid
            else:
                hi = mid
                best = (10.0 ** mid, n)
            if best and abs(best[1] - target) < 0.02 * target:
                break
        return best[0]


def timed_cycles(w, C1, nu, steps, warmup):
    torch, cs = w.torch, w.cs
    stream = cs.stream
    C2 = math.exp(-8.0) * C1
    for k in range(warmup):
        cs.step(nu)
        cs.adapt(C1, C2)
        cs.remap(2)
        log(f"warmup cycle {k} done, {cs.nleaves()} leaves")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    updates = 0
    node_launches = 0
    leaves = []
    cs.profile(True)          # HIP events around every kernel group, on the library's stream
    e0.record(stream)
    for k in range(steps):
        nv = cs.nleaves()
        leaves.append(nv)
        cs.step(nu)
        cs.adapt(C1, C2)
        cs.remap(2)
        updates += w.nc * nv * nu
    e1.record(stream)
    torch.cuda.synchronize()
    prof = cs.profile_read()
    cs.profile(False)
    ms = e0.elapsed_time(e1)
    log(f"timed {steps} cycles: {ms:.1f} ms, leaves {leaves}")
    return updates, ms, leaves, prof


def sweep_only(w, nsweep):
    torch, cs = w.torch, w.cs
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nv = cs.nleaves()
    e0.record(cs.stream)
    cs.step(nsweep)
    e1.record(cs.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cs.check()               # a non-physical state in the timed sweeps fails the run
    return w.nc * nv * nsweep / (ms * 1e-3), ms / nsweep, nv


def measured_traffic(tag, kernel):
    """HBM bytes per (cell, leaf) node of ``kernel`` from the rocprofv3
    FETCH_SIZE/WRITE_SIZE summary kept in profiles/, or None when the kernel
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    sha, per = None, {}
    for line in open(path):
        f = line.split()
        if len(f) == 2 and f[0] == "kernel_source_sha256":
            sha = f[1]
        elif len(f) == 6 and f[0] == "traffic_per_node":
            per[f[1]] = float(f[3]) + float(f[5])
    h = hashlib.sha256()
    for name in ("avs_kernels.hip", "avs_internal.h"):
        with open(os.path.join(ROOT, "paper_2212_05645_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    if sha != h.hexdigest():
        return None
    return per.get(kernel)


def measured_copy_bandwidth(torch, nbytes=2 ** 31, reps=5):
    """Read + write GB/s of a plain device-to-device copy on this GPU (the
    practical HBM ceiling the sweep kernels are compared with)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def vdf_bytes_per_node(P, es):
    """Algorithmic HBM bytes per (cell, leaf) node of one launch of each VDF
    kernel, from the minimum traffic of the method: a step reads the VDF
    twice and writes it once (a leaf row of one cell holds P*es bytes).  The
    reconstruction pass owns one read, the update pass one read and the
    write; interface storage is this design's choice, not algorithmic, and
    counts zero.  Per adaptation: the criterion reads the VDF once, the
    remap and its correction each read and write it once."""
    r = P * es
    return {"passA": r, "passC": 2 * r, "face": 0.0, "criterion": r, "remap_gather": 2 * r,
            "remap_correct": 2 * r, "moments": r}


def design_bytes_per_node(P, es, rows_per_cell, fused_face):
    """Bytes per node this design moves at least: the reconstruction writes
    every interface row once, the update reads each once (and, without the
    fused face moments, the face reduction reads each once more)."""
    r = P * es
    out = {"passA": r * (1.0 + rows_per_cell), "passC": r * (2.0 + rows_per_cell)}
    if not fused_face:
        out["face"] = r * rows_per_cell
    return out


def passA_flops_per_node(D, P, slots, interior):
    """Algorithmic floating-point operations of pass A per (cell, leaf) node
    (an add, multiply or divide counts 1, a fused multiply-add 2; compares,
    min/max, selects and conversions count 0).  ``slots`` = faces per cell,
    ``interior`` = interior neighbours per cell; half of the faces are upwind
    of a node on average.
      least-squares gradient   interior * P * (1 + 2D)   difference, D multiply-adds
      face increments          slots * P * (2D - 1)      grad . (x_f - x_i)
      Venkatakrishnan          slots * P * 12            scaled |D2|, c = b^2 + eps^2,
                                                         numerator, denominator, cross products
      per component            P * (5 + D)               scaling, one division, limited gradient
      upwind sign              slots * (2D - 1)          xi . n in FP64
      reconstruction           slots / 2 * (2D + P * 2D) x_f - xi h - x_i, dot product, + phi
      face moments             slots / 2 * (D^2 + 7D + 5) |xi|^2, A G, A G xi, the (D+1)D/2 second
                                                         moments, energy weight, energy flux terms"""
    return (interior * P * (1 + 2 * D) + slots * P * (2 * D - 1) + slots * P * 12 + P * (5 + D)
            + slots * (2 * D - 1) + slots / 2 * (2 * D + P * 2 * D) + slots / 2 * (D * D + 7 * D + 5))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample_worker(job):
    """One oracle step of a block of cells of the cylinder workload with the
    given leaf set (run in a child process, one thread, BLAS included).
    Returns (updates, t_start, t_end) on the wall clock."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import avs_oracle as O
    from workloads import fields as F
    from workloads import meshes
    nr, nth, first, ncell, level, idx, barrier = job
    c = F.cylinder(nr=nr, nth=nth)
    sample = list(range(first, first + ncell))
    sub, keep = meshes.submesh(c['mesh'], sample, halo=2)
    o = O.Solver(sub, c['vspace'], c['gas'], c['dt'], c['venkat_K'], c['prim0'][keep])
    o.tree = O.Tree(2, o.tree.lo, o.tree.hi, o.tree.base, o.tree.max_level, np.asarray(level, np.int64),
                    np.asarray(idx, np.int64))
    o.phi = o.initial_vdf(o.W)
    loc = [int(np.searchsorted(keep, g)) for g in sample]
    with threadpool_limits(limits=1):
        if barrier is not None:
            barrier.wait(timeout=300)      # a process that failed before this point ends the wait
        t0 = time.time()
        O.step(o.mesh, o.tree, o.gas, o.dt, o.Kv, o.phi, o.W, cells=loc)
        t1 = time.time()
    return len(sample) * len(level), t0, t1


def _proc_job(job, queue):
    try:
        queue.put(_oracle_sample_worker(job))
    except Exception as e:          # reported by the parent
        queue.put(repr(e))


def cpu_baseline(w, args, ncell_sample=256, workers=None):
    """The oracle (FP64 NumPy, as it stands) stepping blocks of cells of the
    same workload and leaf set, given their two-ring neighbourhood, on the
    host: one process on one thread, then one process per core (up to 16,
    the host share of one GPU) each on its own block, all started together
    behind a barrier.  Rates are cell-node updates per second of wall time."""
    import multiprocessing as mp
    L = w.cs.leaves()
    level, idx = L['level'].tolist(), L['idx'].tolist()
    nth = args.nth
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nw = workers or max(1, min(16, ncpu))
    # blocks spread over the radial range (shock layer, wake, far field), all of one size
    firsts = [((w.nc // 2 + k * (w.nc // (2 * nw))) // nth) * nth + (k * 37) % nth for k in range(nw)]
    firsts = [min(f, w.nc - ncell_sample) for f in firsts]
    t0 = time.perf_counter()
    u1, a, b = _oracle_sample_worker((args.nr, nth, firsts[0], ncell_sample, level, idx, None))
    one = u1 / (b - a)
    ctx = mp.get_context("spawn")          # child interpreters: nothing of this process's GPU state
    barrier = ctx.Barrier(nw)
    queue = ctx.Queue()
    procs = [ctx.Process(target=_proc_job, args=((args.nr, nth, f, ncell_sample, level, idx, barrier), queue))
             for f in firsts]
    for pr in procs:
        pr.start()
    res = [queue.get(timeout=900) for _ in procs]
    for pr in procs:
        pr.join()
    bad = [r for r in res if isinstance(r, str)]
    if bad:
        raise RuntimeError(f"oracle worker failed: {bad[0]}")
    total = sum(r[0] for r in res)
    span = max(r[2] for r in res) - min(r[1] for r in res)
    allc = total / span
    log(f"cpu baseline: one thread {one:.3e}, {nw} processes {allc:.3e} updates/s "
        f"({time.perf_counter() - t0:.1f} s with set-up)")
    return {"value": allc, "unit": "cell-node updates/s", "cores": nw, "kind": "oracle",
            "sample": f"one explicit FP64 step of {ncell_sample} contiguous cells x {L['n']} leaves of the same "
                      f"workload per process ({nw} processes, one thread each, BLAS limited to one thread, "
                      f"started together; rate over the span of all), NumPy oracle as it stands",
            "one_thread": {"value": one, "cores": 1, "seconds": b - a},
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity": ncpu}}


def run_batched(args):
    """The batched form: 64 seeded independent cases (FP32) advanced by the
    batched kernels through one captured graph per adaptation cycle."""
    import torch
    from paper_2212_05645_amd import avs
    from workloads import fields as F
    specs = F.batch_cases(seed=0, ncase=args.ncase)
    stream = torch.cuda.Stream()
    cases, W0s, bases = [], [], []
    with torch.cuda.stream(stream):
        for c in specs:
            cap = max(256, int(2.5 * c['target_leaves']))
            cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], c['venkat_K'], c['prim0'], precision=avs.AVS_FP32,
                          leaf_capacity=cap, stream=stream)
            L = cs.leaves()
            cases.append(cs)
            W0s.append(cs.get_W())
            bases.append((L['level'].copy(), L['idx'].copy()))

        def tree(i, C1):
            cs, c = cases[i], specs[i]
            cs.set_leaves(*bases[i])
            cs.set_state(None, W0s[i])
            for _ in range(c['vspace']['max_level']):
                try:
                    cs.adapt(C1, math.exp(-8.0) * C1, probes=c['probes'])
                except avs.AvsError as e:
                    if e.status == avs.AVS_E_CAPACITY:
                        return None
                    raise
                cs.remap(2)
            cs.set_state(None, W0s[i])
            return cs.nleaves()
        C1s = []
        for i, c in enumerate(specs):
            lo, hi, best = -9.0, 0.0, None
            for _ in range(12):
                mid = 0.5 * (lo + hi)
                n = tree(i, 10.0 ** mid)
                if n is None or n > c['target_leaves']:
                    lo = mid
                else:
                    hi, best = mid, 10.0 ** mid
            C1s.append(best if best is not None else 10.0 ** hi)
            tree(i, C1s[-1])
        log(f"batched: {len(cases)} cases, leaves {[cs.nleaves() for cs in cases]}")
        batch = avs.Batch(cases)
        chunk = batch.tune()
        log(f"batched: tuned pass-A chunk {chunk}")

        C2s = [math.exp(-8.0) * C1 for C1 in C1s]

        def cycle():
            batch.step(args.nu, graph=True)
            batch.adapt(C1s, C2s)
            batch.remap(2)
        for _ in range(args.warmup):
            cycle()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        updates = 0
        for _ in range(args.steps):
            updates += sum(cs.nc * cs.nleaves() for cs in cases) * args.nu
            cycle()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        batch.check()
        # sweep-only rate of the captured graph
        nodes = sum(cs.nc * cs.nleaves() for cs in cases)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        batch.step(args.nu, graph=True)
        e0.record(stream)
        batch.step(args.nu, graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        sweep_ms = e0.elapsed_time(e1) / args.nu
        batch.check()
        # the same cases one after another through the single-case entry point
        e0.record(stream)
        for cs in cases:
            cs.step(args.nu)
        e1.record(stream)
        torch.cuda.synchronize()
        seq_ms = e0.elapsed_time(e1) / args.nu
        for cs in cases:
            cs.check()
        # one more cycle with a wait after each phase: adaptation, remap, the
        # first step after it (graph capture + run), a replayed step
        torch.cuda.synchronize()
        t = [time.perf_counter()]
        batch.adapt(C1s, C2s)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        batch.remap(2)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        for _ in range(2):
            batch.step(args.nu, graph=True)
            torch.cuda.synchronize()
            t.append(time.perf_counter())
        batch.check()
        phases = {"adapt_ms": 1e3 * (t[1] - t[0]), "remap_ms": 1e3 * (t[2] - t[1]),
                  "first_steps_ms": 1e3 * (t[3] - t[2]), "replayed_steps_ms": 1e3 * (t[4] - t[3]),
                  "sweeps": args.nu}
        log(f"batched phases: {phases}")
        batch.close()
    return {"cycle_updates_per_s": updates / (ms * 1e-3), "sweep_updates_per_s": nodes / (sweep_ms * 1e-3),
            "sweep_ms": sweep_ms, "sequential_sweep_updates_per_s": nodes / (seq_ms * 1e-3),
            "sequential_sweep_ms": seq_ms, "cases": len(cases), "cell_leaf_nodes": nodes,
            "tuned": {"passA_chunk_per_bucket": chunk[:4], "passC_leaves_in_flight": chunk[4]},
            "roofline_sweep": {"algorithmic_bytes_per_node": 24, "frac": 24 * nodes / (sweep_ms * 1e-3) / HBM_PEAK},
            "cycles_timed": args.steps, "phases": phases,
            "workload": "64 seeded cavity/cylinder cases, Kn 1e-3..1, Ma 0.1..6, grids 32^2..96^2, "
                        "256..16k leaves, FP32, one graph per adaptation cycle"}


def run_learned(args, w, C1):
    """The learned proposal on the same workload: collect plain-criterion
    labels while the case runs, train the network with the library's
    kernels, then time adaptation cycles that use the judged proposal."""
    import numpy as np
    import torch
    from paper_2212_05645_amd import learned
    avs, cs = w.avs, w.cs
    C2 = math.exp(-8.0) * C1
    base = (w.base_level, w.base_idx)
    w.tree(C1)
    mlp = avs.Mlp(learned.init_params(0), max_batch=16384, rho_ref=1.0, T_ref=1.0, stream=cs.stream)
    ds = learned.Dataset(args.train_rows)
    t0 = time.perf_counter()
    learned.collect(cs, mlp, ds, C1, C2, events=args.train_events, sweeps_between=args.nu // 4, base=base,
                    levels=(0, 1, 2), probes=w.cfg['probes'], exact_restore=False)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    nev = len(ds.events)
    split = ds.events[int(0.9 * nev)][0] if nev > 1 else ds.n
    t0 = time.perf_counter()
    losses = learned.train(mlp, ds, epochs=args.train_epochs, batch=8192, lr=2e-3, seed=0,
                           rows=np.arange(split), log_every=50, balance=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    cm = learned.confusion(mlp, ds, rows=np.arange(split, ds.n))
    log(f"learned: {ds.n} labels in {nev} events ({t_collect:.1f} s), trained {args.train_epochs} epochs on {split} "
        f"rows in {t_train:.2f} s, loss {losses[0]:.3f} -> {losses[-1]:.4f}, held-out confusion {cm.tolist()}")
    # timed cycles: plain adaptation, then the learned proposal, from the same step-0 tree
    out = {}
    for mode in ("plain", "learned"):
        w.tree(C1)
        fallbacks, t_adapt, updates = 0, 0.0, 0
        for k in range(args.warmup + args.steps):
            timed = k >= args.warmup
            nv = cs.nleaves()
            if k == args.warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            cs.step(args.nu)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            if mode == "plain":
                cs.adapt(C1, C2)
            else:
                _, _, fb = cs.adapt_learned(mlp, C1, C2, tail_tol=1e-4)
                fallbacks += int(fb and timed)
            tb = time.perf_counter()
            cs.remap(2)
            if timed:
                t_adapt += tb - ta
                updates += w.nc * nv * args.nu
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[mode] = dict(cycle_updates_per_s=updates / (ms * 1e-3), adapt_ms=1e3 * t_adapt / args.steps,
                         fallbacks=fallbacks, leaves=cs.nleaves())
        log(f"learned form, {mode} adaptation: {out[mode]}")
    recall = [float(cm[i, i] / max(cm[i].sum(), 1)) for i in range(3)]
    flop = 3 * 2 * (32 * 128 + 128 * 128 + 128 * 16) * split * args.train_epochs
    mlp.close()
    return {"cycle_updates_per_s": out["learned"]["cycle_updates_per_s"],
            "cycle_updates_per_s_plain_same_run": out["plain"]["cycle_updates_per_s"],
            "adapt_ms_learned": out["learned"]["adapt_ms"], "adapt_ms_plain": out["plain"]["adapt_ms"],
            "fallbacks": out["learned"]["fallbacks"], "cycles": args.steps,
            "leaves_after": {m: out[m]["leaves"] for m in out},
            "labels": ds.n, "train_rows": split, "train_s": t_train, "collect_s": t_collect,
            "train_TFLOP_per_s": flop / t_train / 1e12,
            "heldout_confusion_keep_split_merge": cm.tolist(), "heldout_recall": recall,
            "loss_first_last": [losses[0], losses[-1]]}


def run_initial_avs(args, Ma=5.0, C1=1e-3):
    """The automatic velocity space of Sec. 3.5 on the cylinder mesh at Ma 5:
    host parameters (avs_auto_params), then the step-0 build (uniform
    splits, one probes-only adaptation, closed Maxwellian of W on the new
    leaves, avs_initial_avs), timed end to end.  C1 = 1e-3 suits the
    criterion as printed (the fit of Eq. C1_Ma never splits)."""
    import torch
    from paper_2212_05645_amd import avs
    from workloads import fields as F
    c = F.cylinder(nr=args.nr, nth=args.nth)
    flow = dict(dim=2, R=c['gas']['R'], gamma=5.0 / 3.0, Ma=Ma, T_inf=1.0, T_wall=1.0)
    t0 = time.perf_counter()
    params, vs = avs.auto_params(**flow)
    t_params = time.perf_counter() - t0
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], leaf_capacity=vs['leaf_capacity'])
    cs.initial_avs(C1, params['k_sigma'] * C1, **flow)      # warm-up (first launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = cs.initial_avs(C1, params['k_sigma'] * C1, **flow)
    t_build = time.perf_counter() - t0
    cs.close()
    return {"params_ms": t_params * 1e3, "initial_avs_ms": t_build * 1e3, "leaves": n, "cells": int(c['mesh']['ncells']),
            "L_max": params['L_max'], "L_min": params['L_min'], "L_w": params['L_w'], "R_dv": params['R_dv'],
            "C1": C1, "workload": f"cylinder O-grid {args.nr}x{args.nth}, Ma {Ma}, automatic velocity space (Sec. 3.5)"}


def run_wedge(args, precision, C1=1e-3):
    """Unstructured physical mesh: the hypersonic blunt wedge (Ma 8.1,
    about 11 900 triangles), automatic velocity space of Sec. 3.5 with its
    step-0 build, then the timed cycles of the main workload (sweeps,
    adaptation on cells, closed remap).  C1 = 1e-3 gives a step-0 space of
    574 leaves (the paper's wedge run ends with 568 elements)."""
    import torch
    from paper_2212_05645_amd import avs
    from workloads import fields as F
    flow = F.wedge_flow()
    params, vs = avs.auto_params(**flow)
    c = F.blunt_wedge(vs)
    C2 = params['k_sigma'] * C1
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], leaf_capacity=vs['leaf_capacity'],
                  precision=avs.AVS_FP32 if precision == "fp32" else avs.AVS_FP64)
    n0 = cs.initial_avs(C1, C2, **flow)
    nu = args.nu
    for _ in range(args.warmup):
        cs.step(nu)
        cs.adapt(C1, C2)
        cs.remap(2)
    torch.cuda.synchronize()
    cs.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    updates = 0
    leaves = []
    e0.record(cs.stream)
    for _ in range(args.steps):
        leaves.append(cs.nleaves())
        updates += cs.nc * leaves[-1] * nu
        cs.step(nu)
        cs.adapt(C1, C2)
        cs.remap(2)
    e1.record(cs.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = cs.profile_read()
    cs.profile(False)
    out = {"cycle_updates_per_s": updates / (ms * 1e-3), "ms_per_cycle": ms / args.steps, "cells": cs.nc,
           "leaves_step0": n0, "leaves": leaves, "sweeps_per_cycle": nu, "C1": C1,
           "L_max": params['L_max'], "L_min": params['L_min'], "R_dv": params['R_dv'],
           "kernels_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items()},
           "workload": f"blunt wedge Ma 8.1, unstructured {cs.nc} triangles, automatic velocity space "
                       f"({vs['base'][0]}^2 roots x {vs['max_level']} levels), {precision.upper()}"}
    cs.close()
    return out


def run_implicit_cavity(args, n=64, Kn=6.6e-4, cfl=64.0, macro=60, micro=2, drop=1e-3, max_steps=3000):
    """The implicit step (IUGKS) against the explicit one on a continuum
    lid-driven cavity (n x n cells, Ma 0.16, Kn 6.6e-4, Re 400 by Eq. equ5
    with omega 0.5; 16^2 velocity leaves, FP64): implicit steps at CFL
    ``cfl`` with the paper's sweep counts until the momentum residual has
    dropped by ``drop``, then explicit steps at CFL 0.8 for the same wall
    time.  Reports steps, time per step and the residual each reached."""
    import numpy as np
    import torch
    from paper_2212_05645_amd import avs
    from workloads import fields as F

    def case(c_cfl):
        c = F.cavity(n=n, Kn=Kn, base=8, max_level=1, cfl=c_cfl)
        cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'])
        cs.adapt(-1.0, -2.0)          # every root split once
        cs.remap(2)
        return cs, c['dt']

    ci, dti = case(cfl)
    r0, steps, chunk = None, 0, 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while steps < max_steps:
        r = ci.step_implicit(chunk, macro, micro, residual=True)
        steps += chunk
        rr = float(np.max(r[1:3]))
        r0 = rr if r0 is None else r0
        if rr < drop * r0:
            break
    torch.cuda.synchronize()
    t_imp = time.perf_counter() - t0
    imp = {"cfl": cfl, "dt": dti, "steps": steps, "seconds": t_imp, "ms_per_step": 1e3 * t_imp / steps,
           "residual_drop": rr / r0, "macro_sweeps": macro, "micro_sweeps": micro}
    ci.close()
    ce, dte = case(0.8)
    r0e, stepse, chunk = None, 0, 500
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < t_imp:
        r = ce.step(chunk, residual=True)
        stepse += chunk
        rr = float(np.max(r[1:3]))
        r0e = rr if r0e is None else r0e
    torch.cuda.synchronize()
    t_exp = time.perf_counter() - t0
    exp = {"cfl": 0.8, "dt": dte, "steps": stepse, "seconds": t_exp, "ms_per_step": 1e3 * t_exp / stepse,
           "residual_drop": rr / r0e}
    ce.close()
    # the same implicit run with 20 predictor sweeps instead of 60
    ci, _ = case(cfl)
    r0, steps20, chunk = None, 0, 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while steps20 < max_steps:
        r = ci.step_implicit(chunk, 20, micro, residual=True)
        steps20 += chunk
        rr = float(np.max(r[1:3]))
        r0 = rr if r0 is None else r0
        if rr < drop * r0:
            break
    torch.cuda.synchronize()
    t20 = time.perf_counter() - t0
    ci.close()
    imp20 = {"steps": steps20, "seconds": t20, "ms_per_step": 1e3 * t20 / steps20, "residual_drop": rr / r0,
             "macro_sweeps": 20, "micro_sweeps": micro}
    return {"implicit": imp, "implicit_20_sweeps": imp20, "explicit_same_time": exp, "leaves": 256, "cells": n * n,
            "physical_time_ratio": (imp["steps"] * dti) / (exp["steps"] * dte),
            "workload": f"lid-driven cavity {n}x{n}, Ma 0.16, Kn {Kn} (Re 400), 256 leaves, FP64, "
                        f"implicit CFL {cfl:g} with {macro}/{micro} sweeps vs explicit CFL 0.8"}


def run_rykov(args, reps=5):
    """Rykov equilibrium of the diatomic model (G, H, R on every leaf) for
    one seeded state per cell of the cylinder workload, on its step-0 tree,
    FP64: rate and the write bandwidth against the HBM roofline (3 x 8 B
    written per node; the state rows are read once per cell)."""
    import numpy as np
    import torch
    w = Workload(args, "fp64")
    n0 = w.tree(args.C1)
    cs = w.cs
    rng = np.random.default_rng(3)
    nc = cs.nc
    states = np.concatenate([rng.uniform(0.5, 3.0, (nc, 1)), rng.uniform(-2.0, 2.0, (nc, 2)),
                             rng.uniform(0.5, 8.0, (nc, 2)), 0.1 * rng.standard_normal((nc, 4))], axis=1)
    out = cs.rykov_equilibrium(states)          # first launch (allocates the output)
    st = torch.as_tensor(states, device=cs.device)
    from paper_2212_05645_amd import avs
    g = avs.avs_rykov(3.5, 1.0 / 1.55, 0.2354, 0.3049)
    import ctypes as C
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cs.stream)
    for _ in range(reps):
        avs._check(avs.lib.avs_rykov_equilibrium(cs.ctx, C.byref(g), st.data_ptr(), nc, out.data_ptr(),
                                                 out.numel() * out.element_size()))
    e1.record(cs.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nodes = nc * n0
    gbs = 3 * 8 * nodes / (ms * 1e-3) / 1e9
    res = {"ms_per_launch": ms, "nodes": nodes, "leaves": n0, "cells": nc, "node_rate_per_s": nodes / (ms * 1e-3),
           "write_GBps": gbs, "hbm_frac": gbs * 1e9 / HBM_PEAK,
           "workload": f"Rykov equilibrium (G, H, R), cylinder O-grid {args.nr}x{args.nth}, step-0 tree, FP64"}
    del out, st
    del w
    return res


def run_diatomic(args, steps=10):
    """Rykov diatomic steps (2-D FP64, three reduced distributions) on the
    cylinder workload's mesh and step-0 tree: nitrogen-like gas with
    T_r = 0.9 T_t initially; cell-node updates per second, and the time of
    an implicit step with 20 predictor and 2 micro sweeps."""
    import numpy as np
    import torch
    from paper_2212_05645_amd import avs
    w = Workload(args, "fp64")
    n0 = w.tree(args.C1)
    cs = w.cs
    p = w.cfg['prim0']
    prim = np.concatenate([p[:, :3], p[:, 3:4], 0.9 * p[:, 3:4]], axis=1)
    dia = avs.Diatomic(cs, prim)
    dia.step(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cs.stream)
    dia.step(steps)
    e1.record(cs.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # implicit steps (20 predictor / 2 micro sweeps) at the same dt
    e0.record(cs.stream)
    dia.step_implicit(3, 20, 2)
    e1.record(cs.stream)
    torch.cuda.synchronize()
    ms_imp = e0.elapsed_time(e1) / 3
    out = {"updates_per_s": cs.nc * n0 * 1e3 / ms, "ms_per_step": ms, "cells": cs.nc, "leaves": n0,
           "ms_per_implicit_step_20_2": ms_imp,
           "workload": f"Rykov diatomic explicit step, cylinder O-grid {args.nr}x{args.nth}, step-0 tree, FP64"}
    dia.close()
    del w
    return out


def run_sphere(args):
    """The 3-D form: supersonic sphere (64 x 64 x 32 cells), octree of 16^3
    roots and 2 levels, FP32 storage; C1 for a step-0 tree of about 20 000
    leaves (bisected once with the same step-0 cascade)."""
    import torch
    from paper_2212_05645_amd import avs
    from workloads import fields as F
    c = F.sphere()
    cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], c['venkat_K'], c['prim0'], precision=avs.AVS_FP32,
                  leaf_capacity=49152)
    C1, C2 = args.sphere_C1, math.exp(-8.0) * args.sphere_C1
    for _ in range(c['vspace']['max_level']):
        cs.adapt(C1, C2, probes=c['probes'])
        cs.remap(2)
    cs.set_state(None, cs.get_W())
    n0 = cs.nleaves()
    nu = max(1, args.nu // 4)
    for _ in range(args.warmup):
        cs.step(nu)
        cs.adapt(C1, C2)
        cs.remap(2)
    torch.cuda.synchronize()
    cs.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    updates = 0
    e0.record(cs.stream)
    for _ in range(args.steps):
        updates += cs.nc * cs.nleaves() * nu
        cs.step(nu)
        cs.adapt(C1, C2)
        cs.remap(2)
    e1.record(cs.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = cs.profile_read()
    cs.profile(False)
    out = {"cycle_updates_per_s": updates / (ms * 1e-3), "cells": cs.nc, "leaves_step0": n0,
           "leaves_end": cs.nleaves(), "sweeps_per_cycle": nu, "C1": C1,
           "kernels_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items()},
           "workload": "sphere Ma 4, 64x64x32 cells, octree 16^3 roots x 2 levels on [-12,12]^3, FP32"}
    cs.close()
    return out


def roofline_of(w, r, precision, copy_gbps):
    """Roofline object of the dominant sweep kernel of one form (the longest
    mean launch in the timed cycles), from HIP-event times of the library's
    stream; bytes are the method's algorithmic bytes (2 reads + 1 write of
    the VDF per step), the design's own bytes are reported beside them."""
    P, es = 2, (8 if precision == "fp64" else 4)
    prof = r["prof"]
    nv = r["prof_leaves"]
    nodes = w.nc * nv
    kern = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1]} for k, v in prof.items()}
    bpn = vdf_bytes_per_node(P, es)
    fused = "face" not in prof
    dbn = design_bytes_per_node(P, es, w.nf / w.nc, fused)
    for k in kern:
        if bpn.get(k):
            kern[k]["GB/s"] = bpn[k] * nodes / (kern[k]["ms_per_launch"] * 1e-3) / 1e9
        if k in dbn:
            kern[k]["design_GB/s"] = dbn[k] * nodes / (kern[k]["ms_per_launch"] * 1e-3) / 1e9
    sweep_k = [k for k in ("passA", "face", "face_eqflux", "macro", "target", "passC") if k in kern]
    dom = max(sweep_k, key=lambda k: kern[k]["ms_per_launch"])
    t_launch = kern[dom]["ms_per_launch"] * 1e-3
    tpn = measured_traffic(f"cylinder_{precision}", dom)
    traffic = None if tpn is None else tpn * nodes / 1e9
    if dom != "passA":
        k = "passC"
        alg = bpn[k] * nodes
        achieved = alg / (kern[k]["ms_per_launch"] * 1e-3)
        roofline = {"bound": "hbm", "kernel": k, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": traffic,
                    "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "bytes_per_launch": alg, "algorithmic_bytes_per_node": bpn[k],
                    "design_bytes_per_node": dbn.get(k), "dominant_kernel": dom}
    else:
        # the reconstruction pass is bound by vector-ALU issue (the limiter):
        # its roofline is the FP vector peak (packed FP32 is not used, so both
        # forms issue at the FP64 rate: 256 CU x 64 lanes x 2 flop x 2.4 GHz)
        lr = w.cfg['mesh']['face_lr']
        nint = int((lr[:, 1] >= 0).sum())
        slots, interior = (2 * nint + (w.nf - nint)) / w.nc, 2 * nint / w.nc
        fpn = passA_flops_per_node(2, P, slots, interior)
        alg = fpn * nodes
        achieved = alg / t_launch
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / VALU_PEAK, "traffic": traffic,
                    "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "flops_per_launch": alg, "algorithmic_flops_per_node": fpn,
                    "hbm_GBps": kern[dom].get("GB/s"), "dominant_kernel": dom}
    pc = kern["passC"]
    roofline["passC"] = {"algorithmic_bytes_per_node": bpn["passC"], "GB/s": pc["GB/s"],
                         "frac": pc["GB/s"] * 1e9 / HBM_PEAK, "design_bytes_per_node": dbn["passC"],
                         "design_frac": pc["design_GB/s"] * 1e9 / HBM_PEAK,
                         "frac_of_measured_copy": pc["design_GB/s"] / copy_gbps}
    roofline["measured_copy_GBps"] = copy_gbps
    # the whole sweep (every kernel of one step) against the method's minimum
    # bytes (read the VDF twice, write it once) and against this design's
    sweep_s = sum(kern[k]["ms_per_launch"] for k in sweep_k) * 1e-3
    design_b = sum(dbn.get(k, 0.0) for k in sweep_k)
    min_b = 3 * P * es
    roofline["sweep"] = {"ms": sweep_s * 1e3, "kernels": sweep_k, "algorithmic_bytes_per_node": min_b,
                         "frac": min_b * nodes / sweep_s / HBM_PEAK, "target_frac": 0.60,
                         "design_bytes_per_node": design_b, "design_frac": design_b * nodes / sweep_s / HBM_PEAK}
    return roofline, kern


def run_form(args, precision, C1=None):
    w = Workload(args, precision)
    if C1 is None:
        C1 = w.calibrate(args.leaves) if args.calibrate else args.C1
    n0 = w.tree(C1)
    log(f"{precision}: C1={C1:.6g}, step-0 tree {n0} leaves")
    updates, ms, leaves, prof = timed_cycles(w, C1, args.nu, args.steps, args.warmup)
    sw = sweep_only(w, args.nu) if not args.no_sweep else (None, None, None)
    # kernels of the sweep run once per sweep at the leaf count of their cycle
    mean_leaves = sum(leaves) / len(leaves)
    return w, C1, dict(updates=updates, ms=ms, leaves=leaves, sweep_rate=sw[0], sweep_ms=sw[1], sweep_leaves=sw[2],
                       prof=prof, prof_leaves=mean_leaves)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding over several GPUs is "
              f"designed but not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe > 0:
        n = int(args.copy_probe * 2 ** 30)
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only:
        if args.only == "sphere":
            rec = run_sphere(args)
        elif args.only == "batched":
            rec = run_batched(args)
        else:
            w, C1, _ = run_form(args, "fp64")
            rec = run_learned(args, w, C1)
        print(json.dumps({"form": args.only, **rec}, default=float), flush=True)
        return
    copy_gbps = measured_copy_bandwidth(torch)
    w, C1, r = run_form(args, args.precision)
    roofline, kern = roofline_of(w, r, args.precision, copy_gbps)
    value = r["updates"] / (r["ms"] * 1e-3)
    forms = {args.precision: {"cycle_updates_per_s": value, "sweep_updates_per_s": r["sweep_rate"],
                              "sweep_ms": r["sweep_ms"], "leaves": r["sweep_leaves"]}}
    if args.forms and args.precision == "fp64":
        try:
            forms["learned_fp64"] = run_learned(args, w, C1)
        except Exception as e:
            forms["learned_fp64"] = {"error": repr(e)}
    if not args.one_form:
        # the other precision on the same workload and thresholds, in this run
        other = "fp32" if args.precision == "fp64" else "fp64"
        del w
        torch.cuda.empty_cache()
        w2, _, r2 = run_form(args, other, C1=C1)
        roof2, kern2 = roofline_of(w2, r2, other, copy_gbps)
        forms[other] = {"cycle_updates_per_s": r2["updates"] / (r2["ms"] * 1e-3), "sweep_updates_per_s": r2["sweep_rate"],
                        "sweep_ms": r2["sweep_ms"], "leaves": r2["sweep_leaves"], "ms_per_step": r2["ms"] / args.steps,
                        "roofline": {"frac": roof2["frac"], "kernel": roof2["kernel"], "bound": roof2["bound"],
                                     "passC": roof2["passC"], "sweep": roof2["sweep"]},
                        "kernels": {k: v["ms_per_launch"] for k, v in kern2.items()}}
        f32, f64 = forms.get("fp32"), forms.get("fp64")
        forms["fp32_over_fp64"] = {"cycle": f32["cycle_updates_per_s"] / f64["cycle_updates_per_s"],
                                   "sweep": f32["sweep_updates_per_s"] / f64["sweep_updates_per_s"]}
        w = w2
        del w2
        torch.cuda.empty_cache()
    # the batched form (64 seeded cases, FP32) in every run, a few cycles
    try:
        if args.no_batched:
            raise RuntimeError("skipped (--no-batched)")
        bargs = argparse.Namespace(**vars(args))
        if not args.forms:
            bargs.steps, bargs.warmup = min(args.steps, 3), 1
        b = run_batched(bargs)
        b["over_fp64_sweep"] = b["sweep_updates_per_s"] / forms["fp64"]["sweep_updates_per_s"] if "fp64" in forms else None
        forms["batched_fp32"] = b
    except Exception as e:
        forms["batched_fp32"] = {"error": repr(e)}
    torch.cuda.empty_cache()
    if args.forms:
        try:
            forms["sphere_fp32"] = run_sphere(args)
        except Exception as e:
            forms["sphere_fp32"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            forms["initial_avs"] = run_initial_avs(args)
        except Exception as e:
            forms["initial_avs"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            forms["wedge_unstructured"] = run_wedge(args, args.precision)
        except Exception as e:
            forms["wedge_unstructured"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            forms["implicit_cavity"] = run_implicit_cavity(args)
        except Exception as e:
            forms["implicit_cavity"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            forms["rykov_equilibrium"] = run_rykov(args)
        except Exception as e:
            forms["rykov_equilibrium"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            forms["diatomic_step"] = run_diatomic(args)
        except Exception as e:
            forms["diatomic_step"] = {"error": repr(e)}
    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(w, args)
        except Exception as e:  # the baseline is informative only
            cpu = {"error": repr(e)}
    out = {
        "metric": METRIC, "value": value, "unit": "cell-node updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms"] / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (seeded bow-shock state; no flow data available)",
        "config": {"workload": f"cylinder Ma 5, O-grid {args.nr}x{args.nth}, quadtree 32^2 roots x 3 levels on "
                               f"[-15,15]^2, C1={C1:.4g}, {args.nu} sweeps + adapt + remap per step",
                   "cells": w.nc, "leaves": r["leaves"], "precision": args.precision},
        "roofline": roofline, "cpu_baseline": cpu, "forms": forms, "kernels": kern,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
