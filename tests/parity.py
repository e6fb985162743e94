"""Helpers of the GPU-vs-oracle parity tests: run one workload through the
C ABI (via the ctypes binding) and through the CPU oracle on the same seeded
inputs, then compare element by element.

Tolerances, each derived from the arithmetic it bounds:
  FP64  STATEs   |gpu - ref| <= 1e-12 |ref| + 1e-300 (cable mode: + 5e-11, the
                 v bar times the steepest gate slope 0.05/mV)
        rhs, d   |gpu - ref| <= 1e-11 S_n
        v (isolated compartments, cable) |gpu - ref| <= 1e-9 mV + 1e-12 |ref|:
                 the rhs bar over 1e-3 cm/dt + d >= 0.04 S/cm2 injects about
                 1e-9 mV per step, which the membrane's leak contracts
  FP32  gates and synapse states (nS)   |gpu - ref| <= 1e-5
        cai, cab (free and bound calcium) |gpu - ref| <= 1e-4 |ref|
        rhs, d   |gpu - ref| <= 2e-3 S_n
  node index handling and event decisions: exact (spike counts bit-exact in
  FP64).
S_n = sum over the node's instances of |s| (|i| + 200 mV |g|), an upper bound
of the magnitude of the terms that cancel in rhs and of the finite
difference's numerator scaled by dv.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from oracle import oracle as O

STATE_TOL = {"fp64": (1e-12, 0.0), "fp32": (0.0, 1e-5)}   # (rel, abs)
CAI_REL = {"fp64": 1e-12, "fp32": 1e-4}
NODE_TOL = {"fp64": 1e-11, "fp32": 2e-3}


EPS = 2.0 ** -52
_RECORD = []


def record(label: str, key: str, prec: str, ratio: float, err: float, **extra):
    """Keeps one comparison's worst ratio and error; written out at the end of
    the session when PARITY_RECORD names a file (the calibration of the bars)."""
    test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
    _RECORD.append({"test": test, "label": label, "key": key, "prec": prec, "ratio": ratio, "err": err, **extra})


def dump_record(path: str):
    with open(path, "w") as f:
        json.dump(_RECORD, f)


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(w, nsteps, path="batched", prec="fp64", k0=0, launch=None, vmode=None, unit_nodes=0,
            resident_steps=None):
    """Runs nsteps steps through the C ABI.  The run is split before its
    last step (a split run gives the same bits as one call): the STATEs, v
    and node calcium that the last current update reads are kept under
    "snap", so that rhs and d can be checked against the oracle's current
    update at exactly those inputs (compare_nodes)."""
    from paper_1905_02241_amd import mech
    m = mech.from_workload(w, prec, unit_nodes=unit_nodes)
    if launch is not None:
        m.set_launch(*launch)
    if resident_steps is not None:
        m.set_resident_steps(resident_steps)
    vm = vmode or w.vmode
    if nsteps > 1:
        m.step(nsteps - 1, k0, w.dt, vm, path)
    snap = {"states": mech.states_of(m), "v": m.nodes()["v"], "k": k0 + nsteps - 1, "vmode": vm}
    if nsteps <= 1 and vm == "clamp":
        snap["v"] = None   # the step itself sets v to the clamp value first
    if w.globals.get("shared_ca"):
        snap["cai"] = m.ion("cai")
    m.step(1, k0 + nsteps - 1, w.dt, vm, path)
    m.sync()
    out = {"states": mech.states_of(m), **m.nodes(), "spikes": m.spike_counts(), "snap": snap}
    return out, m


def run_oracle(w, nsteps, k0=0):
    M = O.Model(w)
    M.init()
    M.run(k0, nsteps)
    return M


def oracle_threads() -> int:
    """Threads for the sharded oracle: the usable cores, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run_oracle_sharded(w, nsteps, parts=None, k0=0):
    """The oracle on a workload whose nodes are independent (clamp or
    isolated mode): its nodes cut into contiguous ranges, each range run by
    the single-threaded oracle in its own thread (the oracle keeps no global
    state; its calls release the interpreter lock).  Returns a Model of the
    whole workload holding the merged results, bit-identical to one
    single-threaded run (every node's arithmetic is the same)."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1905_02241_amd import workloads as W
    if w.vmode not in ("clamp", "isolated"):
        raise ValueError("sharding needs independent nodes (clamp or isolated mode)")
    parts = min(parts or oracle_threads(), max(1, w.n_nodes))
    cuts = [c for c in np.array_split(np.arange(w.n_nodes), parts) if c.size]
    shards = [W.subset(w, c) for c in cuts]

    def go(sh):
        M = O.Model(sh[0])
        M.init()
        M.run(k0, nsteps)
        return M

    with ThreadPoolExecutor(len(shards)) as ex:
        runs = list(ex.map(go, shards))
    full = O.Model(w)
    full.init()
    for (sub, keep), Ms, c in zip(shards, runs, cuts):
        for key in ("v", "rhs", "d", "spikes", "cai_node", "ica_node"):
            getattr(full, key)[c] = getattr(Ms, key)
        for s in range(len(w.slots)):
            for name, arr in Ms.states[s].items():
                full.states[s][name][keep[s]] = arr
            full.ica[s][keep[s]] = Ms.ica[s]
    return full


def node_scale(M) -> np.ndarray:
    """S_n from the oracle's final states and voltages."""
    S = np.zeros(M.n_nodes)
    for s, sl in enumerate(M.w.slots):
        node = np.asarray(sl.node)
        for i in range(sl.n):
            n = node[i]
            I, g = M.instance_current(s, i, M.v[n])
            sc = 1e2 / M.area[n] if sl.kind == "syn" else 1.0
            S[n] += sc * (abs(I) + 200.0 * abs(g))
    return S


# Free voltage (isolated compartments, cable): |v_gpu - v_ref| <= V_ABS mV +
# V_REL |v|; the gates follow v, so their bar there adds V_ABS times the
# steepest gate slope, GATE_SLOPE per mV.
V_ABS = {"fp64": 1e-9, "fp32": 1e-2}
V_REL = 1e-12
GATE_SLOPE = 0.05
CAI_FREE_REL = 1e-11


def compare_states(got, M, prec, keep=None, label="", soft=False):
    """Max violation ratio per state (<= 1 passes).  soft: return the
    failures with the ratios instead of asserting."""
    worst = {}
    rel, ab = STATE_TOL[prec]
    for s, sl in enumerate(M.w.slots):
        for name, ref in M.states[s].items():
            g = got["states"][s][name]
            if keep is not None:
                g = g[keep[s]]
            if name in ("cai", "cab"):
                tol = CAI_REL[prec] * np.abs(ref)
                if M.w.vmode in ("cable", "isolated") and prec == "fp64":
                    # the pool integrates its calcium current over tau_ca/dt
                    # (3200) steps, each carrying the gates' v-driven error
                    tol = CAI_FREE_REL * np.abs(ref)
            else:
                tol = rel * np.abs(ref) + ab + 1e-300
                if M.w.vmode in ("cable", "isolated") and prec == "fp64":
                    # gates follow v: the v bar times the steepest gate slope
                    tol = tol + GATE_SLOPE * V_ABS[prec]
            err = np.abs(g - ref)
            r = float(np.max(err / tol)) if err.size else 0.0
            worst[f"{s}:{sl.kind}.{name}"] = (r, float(err.max()) if err.size else 0.0)
            rel_err = float(np.max(err / np.maximum(np.abs(ref), 1e-300))) if err.size else 0.0
            record(label, f"{sl.kind}.{name}", prec, r, worst[f"{s}:{sl.kind}.{name}"][1], rel=rel_err,
                   vmode=M.w.vmode)
    bad = {k: v for k, v in worst.items() if not v[0] <= 1.0}
    if soft:
        return worst, [f"{label} state parity: {bad}"] if bad else []
    assert not bad, f"{label} state parity: {bad}"
    return worst


EPS32 = 2.0 ** -23
FX_RES = 2.0 ** -67   # resolution of the fused paths' fixed-point node sums


def cur_reference(w, snap, nodes=None, keep=None):
    """The oracle's current update (events of step k, then cur) at the
    GPU's own inputs: its STATEs, v and node calcium before that update.
    Returns the oracle model (rhs, d) and its rounding scales."""
    Mr = O.Model(w)
    Mr.init()
    for s in range(len(w.slots)):
        for name, arr in Mr.states[s].items():
            g = snap["states"][s][name]
            arr[:] = g if keep is None else g[keep[s]]
    if snap["v"] is None:
        Mr.vclamp(snap["k"] * w.dt)
    else:
        Mr.v[:] = snap["v"] if nodes is None else snap["v"][nodes]
    if "cai" in snap:
        Mr.cai_node[:] = snap["cai"] if nodes is None else snap["cai"][nodes]
    Mr.events(snap["k"])
    Mr.cur()
    return Mr, Mr.node_scales()


def node_bars(prec, terms, gsum, cnt, dv):
    """Tolerances of rhs and d computed from the same inputs on both sides.
    rhs: each instance current is a short product-and-sum (about seven
    roundings, plus a library exp or log that may differ by an ulp on each
    side), bounded by 8 eps of the magnitudes of its terms; the oracle's
    sequential sum of cnt terms adds (cnt - 1)/2 eps of the same magnitudes
    and the GPU's single rounding of its exact fixed-point total one more.
    d: the finite difference (I(v + dv) - I(v))/dv cancels, so the two
    evaluations' errors enter as 2 * 8 eps T/dv; its own division and the
    sum add (2 + cnt/2) eps of sum |s g|.  FP32-mixed forms the conductance
    products from FP32 STATEs in FP32 (and adds synaptic events in FP32): 8
    float ulps of the products' magnitudes on top.  The fused paths add the
    contributions as fixed-point numbers with 67 fraction bits: each one
    smaller than 2^-15 in magnitude is rounded by at most 2^-68, so cnt
    times 2^-67 is added to both bars."""
    res = cnt * FX_RES
    rhs = EPS * (8.0 + (cnt + 1) / 2.0) * terms + res
    d = EPS * (16.0 * terms / dv + (2.0 + cnt / 2.0) * gsum) + res
    if prec == "fp32":
        rhs = rhs + 8.0 * EPS32 * terms
        d = d + 8.0 * EPS32 * (gsum + terms)
    return rhs + 1e-300, d + 1e-300


def compare_nodes(got, M, prec, nodes=None, label="", check_v=True, keep=None, soft=False):
    """rhs and d, and v along the trajectory.  With the GPU's inputs of its
    last current update (run_gpu's "snap") rhs and d are compared with the
    oracle's current update at those same inputs (node_bars); without them,
    with the oracle's own trajectory at the looser S_n bar.  soft: return
    the failures instead of asserting."""
    out = {}
    fails = []

    def check(ok, msg):
        if soft:
            if not ok:
                fails.append(msg)
        else:
            assert ok, msg
    snap = got.get("snap")
    if snap is not None:
        Mr, (terms, gsum, cnt) = cur_reference(M.w, snap, nodes=nodes, keep=keep)
        bars = node_bars(prec, terms, gsum, cnt, float(M.w.globals["fd_dv"]))
        scales = (terms, gsum + terms / float(M.w.globals["fd_dv"]))
        for key, tol, sc in zip(("rhs", "d"), bars, scales):
            g = got[key] if nodes is None else got[key][nodes]
            ref = getattr(Mr, key)
            err = np.abs(g - ref)
            r = float(np.max(err / tol)) if ref.size else 0.0
            out[key] = r
            units = float(np.max(err / (EPS * sc + 1e-300))) if ref.size else 0.0
            record(label, key, prec, r, float(np.max(err)) if ref.size else 0.0, eps_T=units, vmode=M.w.vmode,
                   same_inputs=True)
            check(r <= 1.0, f"{label} {key} parity ratio {r} (same inputs)")
    else:
        S = node_scale(M)
        for key in ("rhs", "d"):
            g = got[key] if nodes is None else got[key][nodes]
            ref = getattr(M, key)
            tol = NODE_TOL[prec] * S + 1e-300
            r = float(np.max(np.abs(g - ref) / tol)) if ref.size else 0.0
            out[key] = r
            units = float(np.max(np.abs(g - ref) / (EPS * S + 1e-300))) if ref.size else 0.0
            record(label, key, prec, r, float(np.max(np.abs(g - ref))) if ref.size else 0.0, eps_S=units,
                   vmode=M.w.vmode)
            check(r <= 1.0, f"{label} {key} parity ratio {r}")
    if check_v:
        g = got["v"] if nodes is None else got["v"][nodes]
        if M.w.vmode in ("isolated", "cable"):
            tol = V_ABS[prec] + V_REL * np.abs(M.v)
        else:
            tol = (1e-12 if prec == "fp64" else 1e-4) * (np.abs(M.v) + 1.0)
        r = float(np.max(np.abs(g - M.v) / tol)) if M.v.size else 0.0
        out["v"] = r
        record(label, "v", prec, r, float(np.max(np.abs(g - M.v))) if M.v.size else 0.0, vmode=M.w.vmode)
        check(r <= 1.0, f"{label} v parity ratio {r}")
    return (out, fails) if soft else out


class Timer:
    def __enter__(self):
        self.t = time.perf_counter()
        return self

    def __exit__(self, *a):
        self.dt = time.perf_counter() - self.t
