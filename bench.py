"""Throughput of the mechanism path (nrn_cur + nrn_state + voltage provision)
on one MI355X, in mechanism-instance updates per second.

A step is one timestep of every instance of the workload: synapse events,
current update with finite-difference conductance and node reduction,
voltage provision, cnexp state update.  Default workload: 30 M isolated
compartments carrying 40 M hh, 30 M pas, 10 M Ca-HVA + calcium pool and
20 M AMPA/NMDA synapses (about 7.5 GB of algorithmic HBM traffic per FP64
step).  Three variants run on the same inputs: FP64 plain (per-type,
per-phase launches), FP64 batched (one fused launch per step, HIP graphs,
autotuned shape) and FP32-mixed batched.  The headline value is FP64 batched.

Prints progress on stderr and one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per instance per step of the fused step: node index (4,
# none for an identity slot), STATEs read + written, PARAMETERs read,
# ASSIGNED ica written (Ca-HVA); and per node (see node_bytes).  Synapse
# weights are read only on an event.
BYTES_PER_INSTANCE = {
    "fp64": {"pas": 4 + 8 + 8, "hh": 4 + 48 + 24 + 8, "ih": 4 + 16 + 8, "cahva": 4 + 48 + 8 + 8, "syn": 4 + 64},
    "fp32": {"pas": 4 + 4 + 4, "hh": 4 + 24 + 12 + 4, "ih": 4 + 8 + 4, "cahva": 4 + 24 + 4 + 4, "syn": 4 + 32},
}


# Launch shapes of the time-fused path on the default workload (measured
# over block 256/512/1024 and tiles of 512-2048 instances): each tile must
# fit the LDS of a workgroup, and smaller tiles let more of them share a CU.
RESIDENT_SHAPE = {"fp64": (256, 512, 512, 0, 1), "fp32": (512, 2048, 1024, 0, 1)}


def is_identity(slot, n_nodes) -> bool:
    import numpy as np
    return slot.n == n_nodes and bool(np.array_equal(slot.node, np.arange(n_nodes, dtype=slot.node.dtype)))


def node_bytes(w) -> int:
    b = 8 + 8 + 8 + 8            # v read, v written, rhs written, d written
    if w.area is not None and any(s.kind == "syn" for s in w.slots):
        b += 8
    if w.vmode in ("isolated", "cable"):
        b += 8                   # cm
    if w.vmode == "clamp":
        b += 32                  # clamp waveform (off, amp, freq, phase)
    return b


def alg_bytes_per_step(w, prec: str) -> int:
    tot = w.n_nodes * node_bytes(w)
    for s in w.slots:
        tot += s.n * (BYTES_PER_INSTANCE[prec][s.kind] - (4 if is_identity(s, w.n_nodes) else 0))
    return tot


KERNEL_SOURCES = ("mech_kernels.hip", "mech_math.h", "mech_internal.h")


def kernel_source_sha256() -> str:
    """SHA-256 of the kernel sources, concatenated in KERNEL_SOURCES order:
    the key under which profile summaries record what they measured."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1905_02241_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(w, prec: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on the copy probe), or None
    when the summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_fused_{w.name}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha256()
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != sha:
        return None
    v = vals.get(f"traffic_{prec}")
    return None if v in (None, "null") else float(v)


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_variant(w, prec, path, steps, warmup, autotune, torch, mech, launch=None, save_tuning=None,
                 resident=None, plain_atomic=False):
    t0 = time.perf_counter()
    m = mech.from_workload(w, prec)
    torch.cuda.synchronize()
    log(f"{prec}-{path}: context ready in {time.perf_counter() - t0:.1f}s ({m.nbytes / 1e9:.2f} GB)")
    tuned = None
    if path == "plain" and plain_atomic:
        b, t, n, bpc, fl = m.get_launch()
        m.set_launch(b, t, n, bpc, fl | mech.LAUNCH_PLAIN_ATOMIC)
        tuned = {"scatter": "one FP64 atomic per instance"}
    if path == "resident":
        from paper_1905_02241_amd import tuning
        shape, nsub, given = resident
        m.set_resident_steps(nsub)
        cached = tuning.lookup(w, prec, step_path="resident")
        if given:
            m.set_launch(*shape)
            tuned = {"launch": m.get_launch(), "source": "--resident-launch"}
        elif cached is not None and not autotune:
            m.set_launch(*cached)
            tuned = {"launch": m.get_launch(), "source": "tuning cache"}
        elif autotune:
            ms = m.autotune(w.dt, w.vmode, nsteps=nsub, reps=3, path="resident")
            tuned = {"launch": m.get_launch(), "source": "autotuned", "ms_per_step": ms}
            if save_tuning:
                tuning.record(w, prec, m.get_launch(), ms, path=save_tuning, step_path="resident")
        else:
            m.set_launch(*shape)
            tuned = {"launch": m.get_launch(), "source": "default"}
        tuned["steps_per_launch"] = nsub
        log(f"{prec}-{path}: launch {tuned}")
    if path == "batched":
        from paper_1905_02241_amd import tuning
        cached = tuning.lookup(w, prec)
        if launch is not None:
            m.set_launch(*launch)
            tuned = {"launch": m.get_launch(), "source": "--launch"}
        elif cached is not None and not autotune:
            m.set_launch(*cached)
            tuned = {"launch": m.get_launch(), "source": "tuning cache"}
        else:
            ms = m.autotune(w.dt, w.vmode, nsteps=5, reps=3)
            tuned = {"launch": m.get_launch(), "source": "autotuned", "ms_per_step": ms}
            if save_tuning:
                tuning.record(w, prec, m.get_launch(), ms, path=save_tuning)
        log(f"{prec}-{path}: launch {tuned}")
    m.step(warmup, 0, w.dt, w.vmode, path)
    k0 = warmup
    if path == "batched":
        # the batched path replays its middle steps from HIP graphs of at most
        # 64 steps, captured on first use of each length: one untimed call of
        # the timed length captures them before the timed region
        m.step(steps, k0, w.dt, w.vmode, path)
        k0 += steps
    m.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream = m.stream
    torch.cuda.synchronize()
    e0.record(stream)
    m.step(steps, k0, w.dt, w.vmode, path)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    m.sync()
    spikes = int(m.spike_counts().sum()) if w.vmode == "isolated" else None
    info = m.info()
    m.close()
    del m
    torch.cuda.empty_cache()
    ms_step = ms / steps
    ups = w.n_instances / (ms_step * 1e-3)
    gbs = alg_bytes_per_step(w, prec) / (ms_step * 1e-3) / 1e9
    log(f"{prec}-{path}: {ms_step:.4f} ms/step, {ups:.4g} updates/s, {gbs:.0f} GB/s algorithmic")
    out = {"ms_per_step": ms_step, "updates_per_s": ups, "alg_GBps": gbs,
           "alg_bytes_per_step": alg_bytes_per_step(w, prec), "tuned": tuned, "spikes": spikes,
           "tiles": info["n_tiles"]}
    if path == "batched":
        out["launches"] = (f"one fused launch per step; the {steps - 1} middle steps replayed from HIP graphs of at "
                           "most 64 steps, captured before the timed region")
    if path == "resident":
        out["time_fused"] = (f"states stay in LDS for {resident[1]} steps per launch and cross HBM once per "
                             "launch; alg_GBps is the per-step algorithmic bytes over the step time, not HBM "
                             "traffic, and this variant is not the headline")
    return out


def node_sample(w, nodes: int, seed: int):
    """A sample of about `nodes` nodes of the workload as its own workload:
    random nodes, or in cable mode whole cells (the tree solve couples a
    cell's nodes), drawn until the sample is full.  Returns (sub, keep,
    node ids)."""
    import numpy as np
    from paper_1905_02241_amd import workloads as W
    rng = np.random.default_rng(seed)
    if w.vmode == "cable":
        pick, total = [], 0
        for c in rng.permutation(len(w.cell_sizes)):
            if total and total + int(w.cell_sizes[c]) > nodes:
                continue
            pick.append(int(c))
            total += int(w.cell_sizes[c])
        starts = np.concatenate([[0], np.cumsum(w.cell_sizes)])
        ids = np.concatenate([np.arange(starts[c], starts[c + 1]) for c in sorted(pick)])
        sub, keep = W.cells_subset(w, pick)
        return sub, keep, ids
    ids = np.sort(rng.choice(w.n_nodes, size=min(nodes, w.n_nodes), replace=False))
    sub, keep = W.subset(w, ids)
    return sub, keep, ids


def host_cpu():
    """The host's CPU model name (as lscpu reports it) and logical CPU count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def usable_cores(cap: int) -> int:
    """Cores this process may run on, at most `cap` (the CPU share of one
    GPU on a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def node_shards(w, nodes: int, parts: int, seed: int):
    """`parts` disjoint node samples of about `nodes` nodes each, as
    workloads: one sample of parts * nodes nodes cut into contiguous node
    ranges (whole cells in cable mode)."""
    import numpy as np
    from paper_1905_02241_amd import workloads as W
    sub, _, _ = node_sample(w, nodes * parts, seed)
    if w.vmode == "cable":
        sizes = np.asarray(sub.cell_sizes)
        cuts = np.array_split(np.arange(sizes.shape[0]), parts)
        return [W.cells_subset(sub, list(c))[0] for c in cuts if c.size]
    return [W.subset(sub, c)[0] for c in np.array_split(np.arange(sub.n_nodes), parts) if c.size]


def cpu_baseline(w, target_s: float, nodes: int, max_threads: int = 16):
    """The oracle timed on the host: single-threaded on a node sample of the
    same workload (the parity reference as it stands), then one thread per
    usable core, each running the same single-threaded oracle on its own
    disjoint node range of a larger sample (nodes are independent under a
    clamp and in isolated mode, and cells in cable mode; the oracle keeps no
    global state and its calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    sub, _, _ = node_sample(w, nodes, 7)
    M = O.Model(sub)
    M.init()
    t = time.perf_counter()
    M.run(0, 20)
    per = (time.perf_counter() - t) / 20
    steps = int(max(20, min(5000, target_s / max(per, 1e-9))))
    t = time.perf_counter()
    M.run(20, steps)
    dt1 = time.perf_counter() - t
    single = sub.n_instances * steps / dt1
    del M

    threads = usable_cores(max_threads)
    shards = node_shards(w, nodes, threads, 8)
    models = []
    for s in shards:
        m = O.Model(s)
        m.init()
        models.append(m)

    def run(m):
        t0 = time.perf_counter()
        m.run(0, steps)
        return time.perf_counter() - t0

    with ThreadPoolExecutor(len(models)) as ex:
        t = time.perf_counter()
        per_thread = list(ex.map(run, models))
        wall = time.perf_counter() - t
    inst = sum(s.n_instances for s in shards)
    model, ncpu = host_cpu()
    return {"value": inst * steps / wall, "unit": "instance-updates/s", "cores": len(models), "kind": "oracle",
            "sample": f"{len(models)} threads, each the single-threaded FP64 C oracle on its own node range of "
                      f"{inst} instances over {sum(s.n_nodes for s in shards)} nodes of the same workload, "
                      f"{steps} steps, {wall:.1f} s wall (slowest thread {max(per_thread):.1f} s)",
            "single_thread": {"value": single, "cores": 1,
                              "sample": f"{sub.n_nodes} nodes ({sub.n_instances} instances), {steps} steps, "
                                        f"{dt1:.1f} s"},
            "host": {"cpu_model": model, "logical_cpus": ncpu, "usable_cores": usable_cores(10 ** 6)}}


def precision_report(w, steps: int, sample: int, torch, mech):
    """Per-state error of the FP64 and FP32-mixed batched paths against the
    oracle on a node sample after `steps` steps (the precision contract)."""
    import numpy as np
    from oracle import oracle as O
    sub, keep, nodes = node_sample(w, sample, 11)
    M = O.Model(sub)
    M.init()
    M.run(0, steps)
    out = {"steps": steps, "sample_nodes": int(nodes.shape[0]), "vmode": w.vmode}
    for prec in ("fp64", "fp32"):
        m = mech.from_workload(w, prec)
        cached = None
        try:
            from paper_1905_02241_amd import tuning
            cached = tuning.lookup(w, prec)
        except Exception:
            cached = None
        if cached:
            m.set_launch(*cached)
        m.step(steps, 0, w.dt, w.vmode, "batched")
        m.sync()
        st = mech.states_of(m)
        rep = {}
        for s, sl in enumerate(sub.slots):
            for name, ref in M.states[s].items():
                g = st[s][name][keep[s]]
                if ref.size == 0:
                    continue
                err = np.abs(g - ref)
                rel = err / np.maximum(np.abs(ref), 1e-300)
                rep[f"{sl.kind}.{name}"] = {"max_abs": float(err.max()), "max_rel": float(rel.max())}
        v = m.v.cpu().numpy()[nodes]
        rep["v"] = {"max_abs": float(np.max(np.abs(v - M.v)))}
        if w.vmode in ("isolated", "cable"):
            sp = m.spike_counts()[nodes]
            rep["spikes"] = {"match_rate": float(np.mean(sp == M.spikes)), "oracle_total": int(M.spikes.sum()),
                             "gpu_total": int(sp.sum())}
        out[prec] = rep
        m.close()
        log(f"precision {prec}: " + ", ".join(f"{k} {v.get('max_abs', 0):.3g}" for k, v in rep.items()))
    return out


# The precision contract: FP64 STATEs within 1e-12 relative of the oracle;
# FP32-mixed gates and synapse states within 1e-5 absolute, calcium (cai,
# cab, about 5e-5 mM) within 1e-4 relative.
PRECISION_TOL = {"fp64": {"state_rel": 1e-12, "cai_rel": 1e-12},
                 "fp32": {"state_abs": 1e-5, "cai_rel": 1e-4}}


def within_tolerance(rep, prec: str) -> bool:
    """Whether every STATE of a precision report meets its tolerance."""
    tol = PRECISION_TOL[prec]
    for key, e in rep.items():
        if key in ("v", "spikes"):
            continue
        name = key.split(".", 1)[1]
        if name in ("cai", "cab") or prec == "fp64":
            lim = tol["cai_rel"] if name in ("cai", "cab") else tol["state_rel"]
            if not e["max_rel"] <= lim:
                return False
        elif not e["max_abs"] <= tol["state_abs"]:
            return False
    return True


def variant_accuracy(w, settings, steps: int, sample: int):
    """How far a section 5.2 variant (closed-form conductance, Pade cnexp)
    moves the results: the oracle with the variant's globals against the
    oracle without them, per state, on a node sample."""
    import copy
    import numpy as np
    from oracle import oracle as O
    sub, keep, nodes = node_sample(w, sample, 11)
    runs = []
    for on in (False, True):
        s = copy.deepcopy(sub)
        for k, v in settings.items():
            s.globals[k] = v if on else 0
        M = O.Model(s)
        M.init()
        M.run(0, steps)
        runs.append(M)
    exact, var = runs
    out = {"steps": steps, "sample_nodes": int(nodes.shape[0]), "vmode": w.vmode}
    for s, sl in enumerate(sub.slots):
        for name, ref in exact.states[s].items():
            if ref.size == 0:
                continue
            d = np.abs(var.states[s][name] - ref)
            out[f"{sl.kind}.{name}"] = {"max_abs": float(d.max()),
                                        "max_rel": float((d / np.maximum(np.abs(ref), 1e-300)).max())}
    out["v"] = {"max_abs": float(np.max(np.abs(var.v - exact.v)))}
    for key in ("rhs", "d"):
        a, b = getattr(exact, key), getattr(var, key)
        # relative to the largest magnitude on the sample: rhs crosses zero
        out[key] = {"max_abs": float(np.max(np.abs(b - a))),
                    "rel_to_max": float(np.max(np.abs(b - a)) / max(float(np.max(np.abs(a))), 1e-300))}
    if w.vmode in ("isolated", "cable"):
        out["spikes"] = {"match_rate": float(np.mean(var.spikes == exact.spikes)),
                         "exact_total": int(exact.spikes.sum()), "variant_total": int(var.spikes.sum())}
    return out


PROBE_FLAG_SETS = ((), ("nt_load",), ("nt_store",), ("nt_load", "nt_store"), ("8b",), ("chunked",),
                   ("chunked", "nt_store"), ("chunked", "nt_load", "nt_store"))


def probe_battery(mech, nbytes: int = 1 << 32):
    """Every streaming probe at its best unroll (2, 4, 8; 1 to 8 for the
    seven-array probe, 1 to 4 for the twenty-array one) and blocks per CU
    (1, 2, 4, 8, 16): GB/s per op and flag set, with the whole grid."""
    out = {}
    rmw_sets = tuple(fl + extra for fl in ((), ("chunked",), ("nt_load", "nt_store"), ("chunked", "nt_load", "nt_store"))
                     for extra in ((), ("aosoa",))) + (("tiled",), ("tiled", "nt_load", "nt_store"))
    rmw20_sets = ((), ("aosoa",), ("nt_load", "nt_store"), ("aosoa", "nt_load", "nt_store"))
    sets = {"rmw7": rmw_sets, "rmw20": rmw20_sets}
    unrolls = {"rmw7": (1, 2, 4, 8), "rmw20": (1, 2, 4)}
    for op in ("rmw7", "rmw20", "copy", "triad", "split", "read", "write"):
        for fl in sets.get(op, PROBE_FLAG_SETS):
            if op == "read" and "nt_store" in fl or op == "write" and "nt_load" in fl:
                continue
            best, grid = None, {}
            for u in unrolls.get(op, (2, 4, 8)):
                for b in (1, 2, 4, 8, 16):
                    g = mech.probe_stream(op, nbytes, unroll=u, blocks_per_cu=b, reps=5, flags=fl)
                    grid[f"u{u}b{b}"] = round(g)
                    if best is None or g > best[0]:
                        best = (g, u, b)
            key = f"{op}[{'+'.join(fl) or 'plain'}]"
            out[key] = {"GBps": round(best[0], 1), "unroll": best[1], "blocks_per_cu": best[2], "grid": grid}
            log(f"probe {key}: {best[0]:.0f} GB/s (unroll {best[1]}, {best[2]} blocks per CU)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--variants", default="fp64-plain,fp64-batched,fp32-batched,fp64-resident,fp32-resident")
    ap.add_argument("--autotune", action="store_true",
                    help="run the launch-shape autotuner even when the tuning cache has an entry")
    ap.add_argument("--save-tuning", default=None, help="JSON file to record autotuned shapes in")
    ap.add_argument("--no-probe", action="store_true", help="skip the streaming-copy ceiling probe")
    ap.add_argument("--probe-battery", action="store_true",
                    help="instead of timing the workload: every streaming probe (copy, triad, split read/write "
                         "waves, read, write) with and without non-temporal hints, 8-byte accesses and chunked "
                         "mapping, each at its best unroll and blocks per CU")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-steps", type=int, default=1000,
                    help="steps of the per-state error check against the oracle in the bench record (0: skip)")
    ap.add_argument("--precision-nodes", type=int, default=3000,
                    help="node sample of the per-state error check in the bench record")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-nodes", type=int, default=20000)
    ap.add_argument("--precision-report", type=int, default=0, metavar="NODES",
                    help="instead of timing: per-state error of FP64 and FP32-mixed vs the oracle on a node sample")
    ap.add_argument("--vmode", default=None, choices=("clamp", "isolated", "cable"),
                    help="voltage provision instead of the workload's own (cable needs a workload with cell "
                         "trees, config 4)")
    ap.add_argument("--launch", default=None,
                    help="fixed batched launch shape 'block,tile_instances,tile_nodes,blocks_per_cu' (no autotune)")
    ap.add_argument("--resident-launch", default=None,
                    help="launch shape of the time-fused path 'block,tile_instances,tile_nodes,blocks_per_cu,flags' "
                         "(default: the tuning cache, else FP64 256,512,512,0,1 and FP32 512,2048,1024,0,1)")
    ap.add_argument("--resident-steps", type=int, default=64, help="steps per launch of the time-fused path")
    ap.add_argument("--plain-scatter", default="segmented", choices=("segmented", "atomic"),
                    help="scatter of the plain path's current update: the wave-segmented per-node sum (default) "
                         "or one FP64 atomic per instance")
    ap.add_argument("--set", action="append", default=[], metavar="NAME=VALUE",
                    help="set a global of the workload (e.g. pade_cnexp=1, analytic_conductance=1); repeatable")
    ap.add_argument("--variant-accuracy", type=int, default=0, metavar="NODES",
                    help="instead of timing: the oracle with the --set globals against the oracle without them, "
                         "per state, on a node sample (CPU only)")
    args = ap.parse_args()

    settings = {}
    for kv in args.set:
        k, _, v = kv.partition("=")
        settings[k.strip()] = float(v)

    if args.variant_accuracy:
        from paper_1905_02241_amd import workloads as W
        w = W.make_config(args.config, scale=args.scale)
        if args.vmode:
            w.vmode = args.vmode
        rep = variant_accuracy(w, settings, args.steps, args.variant_accuracy)
        print(json.dumps({"variant_accuracy": rep, "workload": w.name, "set": settings}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the mechanism path has no "
              "multi-GPU mode", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_02241_amd import mech, workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    mech.load_library()
    torch.cuda.set_device(0)

    if args.probe_battery:
        print(json.dumps({"probe_battery": probe_battery(mech)}), flush=True)
        return

    t0 = time.perf_counter()
    w = W.make_config(args.config, scale=args.scale)
    if args.vmode:
        if args.vmode == "cable" and getattr(w, "parent", None) is None:
            print(f"workload {w.name} has no cell trees for the cable mode", file=sys.stderr)
            sys.exit(2)
        if args.vmode == "clamp" and w.clamp_off is None:
            print(f"workload {w.name} has no clamp waveform", file=sys.stderr)
            sys.exit(2)
        w.vmode = args.vmode
    for k, v in settings.items():
        w.globals[k] = v
    log(f"workload {w.name}: {w.n_nodes} nodes, {w.instance_counts()}, vmode {w.vmode}, "
        f"built in {time.perf_counter() - t0:.1f}s" + (f", globals set {settings}" if settings else ""))

    if args.precision_report:
        rep = precision_report(w, args.steps, args.precision_report, torch, mech)
        print(json.dumps({"precision_report": rep, "workload": w.name}), flush=True)
        return

    res = {}
    for v in args.variants.split(","):
        prec, path = v.split("-")
        if path == "resident" and w.vmode not in ("clamp", "isolated"):
            log(f"{v}: skipped, the time-fused path runs in clamp and isolated modes only")
            continue
        launch = tuple(int(x) for x in args.launch.split(",")) if args.launch else None
        shape = tuple(int(x) for x in args.resident_launch.split(",")) if args.resident_launch else RESIDENT_SHAPE[prec]
        resident = (shape, args.resident_steps, args.resident_launch is not None)
        res[v] = time_variant(w, prec, path, args.steps, args.warmup, args.autotune, torch, mech, launch,
                              args.save_tuning, resident, args.plain_scatter == "atomic")

    probe = hh_probe = hh_probe_tiles = None
    if not args.no_probe:
        probe = max(mech.probe_stream("copy", 1 << 32, unroll=u, blocks_per_cu=b, flags=fl)
                    for u in (2, 4, 8) for b in (1, 2, 4) for fl in ((), ("nt_load", "nt_store")))
        log(f"copy probe: {probe:.0f} GB/s (read + write, 4 GiB, best of unroll 2/4/8 x 1/2/4 blocks per CU, "
            "with and without non-temporal hints)")
        # the stream of one hh slot (seven FP64 arrays, three rewritten), grid-stride and with one
        # contiguous range per workgroup as the fused kernel's tiles have
        hh_probe, hh_probe_tiles = (
            max(mech.probe_stream("rmw7", 1 << 32, unroll=u, blocks_per_cu=b, flags=fl + extra)
                for u in (1, 4) for b in (1, 4) for fl in ((), ("nt_load", "nt_store")))
            for extra in ((), ("chunked",)))
        log(f"hh-shaped probe: {hh_probe:.0f} GB/s grid-stride, {hh_probe_tiles:.0f} GB/s one range per workgroup")

    head_key = "fp64-batched" if "fp64-batched" in res else next(iter(res))
    head = res[head_key]
    prec = head_key.split("-")[0]
    achieved = head["alg_GBps"]
    out = {
        "metric": "mechanism-instance updates/s (cur+state) + % HBM peak, FP64 plain vs FP32 batched",
        "value": head["updates_per_s"],
        "unit": "instance-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_nodes": w.n_nodes, "instances": w.instance_counts(),
                   "dt_ms": w.dt, "vmode": w.vmode, "path": head_key, "parallelism": "single GPU",
                   **({"globals_set": settings} if settings else {})},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w, prec),
                     "kernel": f"k_fused (state+cur, {w.vmode})",
                     "alg_bytes_per_launch": head["alg_bytes_per_step"],
                     "copy_probe_GBps": probe,
                     "frac_of_copy_probe": (achieved / probe) if probe else None,
                     "hh_stream_probe_GBps": hh_probe,
                     "hh_stream_probe_one_range_per_workgroup_GBps": hh_probe_tiles},
        "variants": res,
    }
    if "fp32-batched" in res and "fp64-plain" in res:
        out["fp32_batched_over_fp64_plain"] = res["fp32-batched"]["updates_per_s"] / res["fp64-plain"]["updates_per_s"]
    if "fp64-batched" in res and "fp64-plain" in res:
        out["fp64_batched_over_fp64_plain"] = res["fp64-batched"]["updates_per_s"] / res["fp64-plain"]["updates_per_s"]
    for pr in ("fp64", "fp32"):
        if f"{pr}-resident" in res and f"{pr}-batched" in res:
            out[f"{pr}_resident_over_{pr}_batched"] = (res[f"{pr}-resident"]["updates_per_s"] /
                                                       res[f"{pr}-batched"]["updates_per_s"])
    if args.precision_steps > 0 and {"fp64-batched", "fp32-batched"} & set(res):
        log(f"precision check: {args.precision_steps} steps, {args.precision_nodes}-node sample ...")
        rep = precision_report(w, args.precision_steps, args.precision_nodes, torch, mech)
        for pr in ("fp64", "fp32"):
            rep[pr]["within_tolerance"] = within_tolerance(rep[pr], pr)
        rep["tolerances"] = PRECISION_TOL
        out["precision"] = rep
        log(f"precision check: fp64 within tolerance {rep['fp64']['within_tolerance']}, "
            f"fp32 within tolerance {rep['fp32']['within_tolerance']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, args.cpu_nodes)
        cb = out["cpu_baseline"]
        log(f"cpu baseline {cb['value']:.4g} updates/s on {cb['cores']} threads, "
            f"{cb['single_thread']['value']:.4g} on one ({cb['host']['cpu_model']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
