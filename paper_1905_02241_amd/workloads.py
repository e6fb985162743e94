"""Seeded synthetic workloads for the mechanism kernels.

This module only draws random numbers and sets constants: it holds none of the
method's arithmetic, so both the GPU library (through ``mech.py``) and the
CPU oracle (through ``oracle/oracle.py``) consume the same inputs without
sharing any code path.

The paper's own models (the somatosensory microcircuit and the hippocampus
CA1 model of section 7) are not available, so every input is synthetic, with
the shapes of section 7's benchmarks: density mechanisms at one instance per
compartment, point-process synapses at several per compartment (the CA1 model
of section 1 has about 6.4 synapses per compartment), dt = 0.025 ms.

Units: mV, ms, S/cm2, um2, uF/cm2, mM, Hz, nS.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

KINDS = ("pas", "hh", "ih", "cahva", "syn", "kmarkov", "capump", "cabuf")
KIND_ID = {k: i for i, k in enumerate(KINDS)}

# Variable names of every mechanism type (interface only).
PARAM_NAMES = {
    "pas": ("g", "e"),
    "hh": ("gnabar", "gkbar", "gl", "el"),
    "ih": ("gbar",),
    "cahva": ("gbar",),
    "syn": ("weight",),
    "kmarkov": ("gbar",),
    "capump": ("gbar",),
    "cabuf": ("gbar",),
}
STATE_NAMES = {
    "pas": (),
    "hh": ("m", "h", "n"),
    "ih": ("m",),
    "cahva": ("m", "h", "cai"),
    "syn": ("A_ampa", "B_ampa", "A_nmda", "B_nmda"),
    "kmarkov": ("C1", "C2", "O"),
    "capump": ("m", "h", "cai"),
    "cabuf": ("m", "h", "cai", "cab"),
}
PARAM_DEFAULTS = {
    "pas": {"g": 1e-3, "e": -70.0},
    "hh": {"gnabar": 0.12, "gkbar": 0.036, "gl": 0.0003, "el": -54.3},
    "ih": {"gbar": 1e-4},
    "cahva": {"gbar": 5e-5},
    "syn": {"weight": 1.0},
    "kmarkov": {"gbar": 0.01},
    "capump": {"gbar": 5e-5},
    "cabuf": {"gbar": 5e-5},
}

DEFAULT_GLOBALS = {
    "celsius": 6.3,
    "ena": 50.0,
    "ek": -77.0,
    "eh": -45.0,
    "cao": 2.0,
    "cai0": 5e-5,
    "tau_ca": 80.0,
    "ca_gamma": 0.05,
    "ca_depth": 0.1,
    "e_syn": 0.0,
    "mg": 1.0,
    "tau_r_ampa": 0.2,
    "tau_d_ampa": 1.7,
    "tau_r_nmda": 0.29,
    "tau_d_nmda": 43.0,
    "event_rate_hz": 5.0,
    "vthresh": -20.0,
    "fd_dv": 1e-3,
    "event_seed": 0,
    "analytic_conductance": 0,   # section 5.2: closed-form di/dv instead of the finite difference
    "pade_cnexp": 0,             # section 5.2: (1,1) Pade approximant of the cnexp exponential
    "pump_vmax": 1e-4,           # capump: maximal pump rate (mM/ms)
    "pump_kp": 1e-3,             # capump: pump half-activation (mM)
    "newton_iters": 4,           # capump: Newton steps per implicit Euler step
    "shared_ca": 0,              # 1: calcium is a per-node ion shared by the calcium channels of a node
    "buf_total": 0.05,           # cabuf: total calcium buffer (mM)
    "buf_kon": 100.0,            # cabuf: binding rate (1/(mM ms)); with buf_koff a 1 uM dissociation constant
    "buf_koff": 0.1,             # cabuf: unbinding rate (1/ms)
}

VMODES = ("external", "clamp", "isolated", "cable")
SEED_BASE = 20190506


@dataclasses.dataclass
class Slot:
    kind: str
    node: np.ndarray                      # int32 [n]
    params: Dict[str, np.ndarray]         # float64 [n] each
    gid: Optional[np.ndarray] = None      # int64 [n] (synapse event-stream id)

    @property
    def n(self) -> int:
        return int(self.node.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    n_nodes: int
    slots: List[Slot]
    vmode: str
    dt: float
    nsteps: int
    v_init: float = -65.0
    area: Optional[np.ndarray] = None      # float64 [n_nodes]
    cm: Optional[np.ndarray] = None        # float64 [n_nodes]
    clamp_off: Optional[np.ndarray] = None
    clamp_amp: Optional[np.ndarray] = None
    clamp_freq: Optional[np.ndarray] = None
    clamp_phase: Optional[np.ndarray] = None
    globals: Dict[str, float] = dataclasses.field(default_factory=lambda: dict(DEFAULT_GLOBALS))
    parent: Optional[np.ndarray] = None    # int32 [n_nodes], cable mode: parent node (-1 root), Hines order
    g_axial: Optional[np.ndarray] = None   # float64 [n_nodes], cable mode: uS to the parent

    @property
    def n_instances(self) -> int:
        return sum(s.n for s in self.slots)

    def instance_counts(self) -> Dict[str, int]:
        out: Dict[str, int] = {}
        for s in self.slots:
            out[s.kind] = out.get(s.kind, 0) + s.n
        return out


# --------------------------------------------------------------- helpers --
def _params(kind: str, n: int, overrides: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    p = {name: np.full(n, PARAM_DEFAULTS[kind][name], dtype=np.float64) for name in PARAM_NAMES[kind]}
    if overrides:
        for k, v in overrides.items():
            p[k] = np.ascontiguousarray(v, dtype=np.float64)
    return p


def _slot(kind: str, node: np.ndarray, params=None, gid=None) -> Slot:
    node = np.ascontiguousarray(node, dtype=np.int32)
    if gid is None and kind == "syn":
        gid = np.arange(node.shape[0], dtype=np.int64)
    return Slot(kind, node, _params(kind, node.shape[0], params),
                None if gid is None else np.ascontiguousarray(gid, dtype=np.int64))


def _sinusoid_clamp(rng: np.random.Generator, n: int):
    """-65 mV offset, amplitude U[30, 60] mV, frequency U[5, 50] Hz, phase U[0, 2 pi)."""
    off = np.full(n, -65.0)
    amp = rng.uniform(30.0, 60.0, n)
    freq = rng.uniform(5.0, 50.0, n)
    phase = rng.uniform(0.0, 2.0 * np.pi, n)
    return off, amp, freq, phase


def _syn_slot(rng: np.random.Generator, n_nodes: int, mean_per_node: float, shuffle: bool) -> Slot:
    counts = rng.poisson(mean_per_node, n_nodes)
    node = np.repeat(np.arange(n_nodes, dtype=np.int32), counts)
    if shuffle:
        node = node[rng.permutation(node.shape[0])]
    w = rng.lognormal(0.0, 0.5, node.shape[0])
    return _slot("syn", node, {"weight": w})


def _globals(cfg_id: int) -> Dict[str, float]:
    g = dict(DEFAULT_GLOBALS)
    g["event_seed"] = 0x5EED0000 + cfg_id
    return g


# -------------------------------------------------------------- configs --
def make_c1(seed: int = SEED_BASE + 0, n_nodes: int = 10_000, nsteps: int = 1000) -> Workload:
    """hh only, one instance per node, each node clamped at a constant
    voltage drawn from U[-80, 40] mV; states start at steady state at -65 mV."""
    rng = np.random.default_rng(seed)
    vc = rng.uniform(-80.0, 40.0, n_nodes)
    z = np.zeros(n_nodes)
    return Workload("hh-10k-clamp", n_nodes, [_slot("hh", np.arange(n_nodes))], "clamp", 0.025, nsteps,
                    clamp_off=vc, clamp_amp=z.copy(), clamp_freq=z.copy(), clamp_phase=z.copy(),
                    globals=_globals(0))


def make_c2(seed: int = SEED_BASE + 1, n_nodes: int = 1_000_000, nsteps: int = 4000) -> Workload:
    """hh + pas at every node (one of each, identity node_index), sinusoidal clamp."""
    rng = np.random.default_rng(seed)
    off, amp, freq, phase = _sinusoid_clamp(rng, n_nodes)
    nodes = np.arange(n_nodes)
    return Workload("hh+pas-1M-clamp", n_nodes, [_slot("pas", nodes), _slot("hh", nodes)], "clamp", 0.025,
                    nsteps, clamp_off=off, clamp_amp=amp, clamp_freq=freq, clamp_phase=phase,
                    globals=_globals(1))


def make_c3(seed: int = SEED_BASE + 2, n_nodes: int = 500_000, nsteps: int = 4000,
            syn_per_node: float = 10.0) -> Workload:
    """AMPA+NMDA synapses, Poisson(10) per node, node_index in random order,
    weights lognormal(0, 0.5) nS, 5 Hz Poisson input, sinusoidal clamp."""
    rng = np.random.default_rng(seed)
    off, amp, freq, phase = _sinusoid_clamp(rng, n_nodes)
    area = rng.uniform(100.0, 1000.0, n_nodes)
    syn = _syn_slot(rng, n_nodes, syn_per_node, shuffle=True)
    return Workload("syn-5M-random", n_nodes, [syn], "clamp", 0.025, nsteps, area=area,
                    clamp_off=off, clamp_amp=amp, clamp_freq=freq, clamp_phase=phase, globals=_globals(2))


def random_cell(rng: np.random.Generator, n: int, first: int, mean_section: float = 8.0,
                ra: float = 100.0):
    """One cell of n compartments in Hines order (parent index < own index),
    numbered from `first`: a soma (diameter 20 um, length 20 um) and
    unbranched sections of 1 + Poisson(mean_section - 1) compartments, each
    attached to a uniformly chosen existing compartment.  Per section a
    diameter U[0.5, 3] um, per compartment a length U[10, 30] um; area
    pi d l (um2) and the axial conductance to the parent 1e2 pi (d/2)^2 /
    (ra l) uS (ra in ohm cm, l in um), computed on the child's geometry."""
    parent = np.empty(n, dtype=np.int32)
    diam = np.empty(n)
    length = np.empty(n)
    parent[0], diam[0], length[0] = -1, 20.0, 20.0
    k = 1
    while k < n:
        m = min(n - k, 1 + int(rng.poisson(mean_section - 1.0)))
        at = int(rng.integers(0, k))
        d = rng.uniform(0.5, 3.0)
        for j in range(m):
            parent[k + j] = first + (at if j == 0 else k + j - 1)
        diam[k:k + m] = d
        length[k:k + m] = rng.uniform(10.0, 30.0, m)
        k += m
    area = np.pi * diam * length
    g = 1e2 * np.pi * (diam / 2.0) ** 2 / (ra * length)
    g[0] = 0.0
    return parent, area, g


def make_c4(seed: int = SEED_BASE + 3, n_cells: int = 64, nsteps: int = 4000,
            lo: int = 200, hi: int = 20_000) -> Workload:
    """64 cells of log-uniform 200..20000 compartments, nodes contiguous per
    cell in Hines order (random branched morphologies, see random_cell);
    pas + hh everywhere, Ih and Ca-HVA on a seeded 30 %, synapses at
    Poisson(3) per compartment; sinusoidal clamp by default, or 'cable' mode
    with the cells' tree coupling."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), n_cells))).astype(np.int64)
    n_nodes = int(sizes.sum())
    off, amp, freq, phase = _sinusoid_clamp(rng, n_nodes)
    nodes = np.arange(n_nodes)
    sub = np.sort(rng.choice(n_nodes, size=int(round(0.3 * n_nodes)), replace=False))
    syn = _syn_slot(rng, n_nodes, 3.0, shuffle=False)
    trng = np.random.default_rng(seed + 1000)
    parts, first = [], 0
    for sz in sizes:
        parts.append(random_cell(trng, int(sz), first))
        first += int(sz)
    parent = np.concatenate([p[0] for p in parts])
    area = np.concatenate([p[1] for p in parts])
    g_axial = np.concatenate([p[2] for p in parts])
    w = Workload("cells64-mixed", n_nodes,
                 [_slot("pas", nodes), _slot("hh", nodes), _slot("ih", sub), _slot("cahva", sub), syn],
                 "clamp", 0.025, nsteps, area=area, cm=np.ones(n_nodes),
                 clamp_off=off, clamp_amp=amp, clamp_freq=freq, clamp_phase=phase, globals=_globals(3),
                 parent=parent, g_axial=g_axial)
    w.cell_sizes = sizes  # type: ignore[attr-defined]
    return w


def make_cells(seed: int, n_cells: int, lo: int, hi: int, kinds=("pas", "hh", "syn"), syn_per_node: float = 2.0,
               event_rate_hz: float = 300.0, nsteps: int = 200, mean_section: float = 8.0) -> Workload:
    """Small branched cells for cable-mode parity tests."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, n_cells)
    parts, first = [], 0
    for sz in sizes:
        parts.append(random_cell(rng, int(sz), first, mean_section))
        first += int(sz)
    n_nodes = first
    parent = np.concatenate([p[0] for p in parts])
    area = np.concatenate([p[1] for p in parts])
    g_axial = np.concatenate([p[2] for p in parts])
    nodes = np.arange(n_nodes)
    slots = []
    for k in kinds:
        if k == "syn":
            s = _syn_slot(rng, n_nodes, syn_per_node, shuffle=True)
            s.params["weight"][:] *= 4.0
            slots.append(s)
        else:
            slots.append(_slot(k, nodes))
    g = _globals(200)
    g["event_seed"] = 0xCAB1E + seed
    g["event_rate_hz"] = event_rate_hz
    w = Workload(f"cells-{seed}", n_nodes, slots, "cable", 0.025, nsteps, area=area, cm=np.ones(n_nodes),
                 globals=g, parent=parent, g_axial=g_axial)
    w.cell_sizes = sizes  # type: ignore[attr-defined]
    return w


def make_c5(seed: int = SEED_BASE + 4, n_nodes: int = 30_000_000, nsteps: int = 10_000) -> Workload:
    """Mixed instances over isolated compartments (free voltage):
    hh at every node plus a second hh on a seeded third of the nodes (sorted,
    many-to-one), pas at every node, Ca-HVA on a seeded third, synapses at
    Poisson(2/3) per node (sorted); 5 Hz input, area U[100, 1000] um2,
    cm = 1 uF/cm2."""
    rng = np.random.default_rng(seed)
    third = n_nodes // 3
    nodes = np.arange(n_nodes, dtype=np.int32)
    hh2 = rng.choice(n_nodes, size=third, replace=False).astype(np.int32)
    hh_node = np.sort(np.concatenate([nodes, hh2]))
    ca_node = np.sort(rng.choice(n_nodes, size=third, replace=False)).astype(np.int32)
    syn = _syn_slot(rng, n_nodes, 2.0 / 3.0, shuffle=False)
    area = rng.uniform(100.0, 1000.0, n_nodes)
    cm = np.ones(n_nodes)
    return Workload("mixed-100M-isolated", n_nodes,
                    [_slot("pas", nodes), _slot("hh", hh_node), _slot("cahva", ca_node), syn],
                    "isolated", 0.025, nsteps, area=area, cm=cm, globals=_globals(4))


_MAKERS = {1: make_c1, 2: make_c2, 3: make_c3, 4: make_c4, 5: make_c5}


def make_config(i: int, scale: float = 1.0, **kw) -> Workload:
    """Config i (1..5); `scale` shrinks node / cell counts for parity tests."""
    if scale != 1.0:
        if i == 4:
            kw.setdefault("n_cells", max(1, int(round(64 * scale))))
        else:
            base = {1: 10_000, 2: 1_000_000, 3: 500_000, 5: 30_000_000}[i]
            kw.setdefault("n_nodes", max(1, int(round(base * scale))))
    return _MAKERS[i](**kw)


# ---------------------------------------------------------- small cases --
def make_tiny(seed: int, kinds=("pas", "hh", "ih", "cahva", "syn"), n_nodes: int = 48,
              per_node: int = 1, syn_per_node: float = 3.0, shuffle: bool = True,
              vmode: str = "clamp", nsteps: int = 50, dt: float = 0.025,
              event_rate_hz: float = 400.0, density_fraction: float = 1.0) -> Workload:
    """Small random mesh for brute-force parity: every density kind sits on a
    random subset of nodes with `per_node` instances each, synapses at
    Poisson(syn_per_node) per node; node_index shuffled if `shuffle`.
    Parameters are randomised around their defaults so no instance is
    special.  The event rate is high so events occur within few steps."""
    rng = np.random.default_rng(seed)
    slots = []
    for kind in kinds:
        if kind == "syn":
            s = _syn_slot(rng, n_nodes, syn_per_node, shuffle)
            slots.append(s)
            continue
        m = max(1, int(round(density_fraction * n_nodes)))
        base = np.sort(rng.choice(n_nodes, size=m, replace=False))
        node = np.repeat(base, per_node)
        if shuffle:
            node = node[rng.permutation(node.shape[0])]
        n = node.shape[0]
        p = {}
        for name in PARAM_NAMES[kind]:
            d = PARAM_DEFAULTS[kind][name]
            if name in ("e", "el"):
                p[name] = d + rng.uniform(-5.0, 5.0, n)
            else:
                p[name] = d * rng.uniform(0.5, 1.5, n)
        slots.append(_slot(kind, node, p))
    off, amp, freq, phase = _sinusoid_clamp(rng, n_nodes)
    area = rng.uniform(100.0, 1000.0, n_nodes)
    cm = rng.uniform(0.8, 1.2, n_nodes)
    g = _globals(100)
    g["event_seed"] = 0x7153 + seed
    g["event_rate_hz"] = event_rate_hz
    return Workload(f"tiny-{seed}", n_nodes, slots, vmode, dt, nsteps, area=area, cm=cm,
                    clamp_off=off, clamp_amp=amp, clamp_freq=freq, clamp_phase=phase, globals=g)


def subset(w: Workload, node_ids: np.ndarray):
    """Restrict a workload to a node sample (nodes are independent under a
    clamp or in isolated mode).  Returns the sub-workload and, per slot, the
    indices of the kept instances in the original slot order.  Synapses keep
    their original event-stream id."""
    node_ids = np.unique(np.asarray(node_ids, dtype=np.int64))
    remap = np.full(w.n_nodes, -1, dtype=np.int64)
    remap[node_ids] = np.arange(node_ids.shape[0])
    slots, keep = [], []
    for s in w.slots:
        idx = np.nonzero(remap[s.node] >= 0)[0]
        gid = None
        if s.kind == "syn":
            gid = (s.gid if s.gid is not None else np.arange(s.n, dtype=np.int64))[idx]
        slots.append(Slot(s.kind, remap[s.node[idx]].astype(np.int32),
                          {k: v[idx].copy() for k, v in s.params.items()}, gid))
        keep.append(idx)

    def pick(a):
        return None if a is None else a[node_ids].copy()

    sub = Workload(w.name + "-sample", int(node_ids.shape[0]), slots, w.vmode, w.dt, w.nsteps, w.v_init,
                   pick(w.area), pick(w.cm), pick(w.clamp_off), pick(w.clamp_amp), pick(w.clamp_freq),
                   pick(w.clamp_phase), dict(w.globals))
    if w.parent is not None:
        # a node sample keeps its tree only if it holds whole cells; otherwise
        # the nodes are cut loose (valid under a clamp or in isolated mode)
        p = w.parent[node_ids]
        inside = (p >= 0) & (remap[np.maximum(p, 0)] >= 0)
        sub.parent = np.where(inside, remap[np.maximum(p, 0)], -1).astype(np.int32)
        sub.g_axial = np.where(inside, w.g_axial[node_ids], 0.0)
    return sub, keep


def cells_subset(w: Workload, cells) -> tuple:
    """Restrict a cell workload to whole cells (cable mode stays valid)."""
    starts = np.concatenate([[0], np.cumsum(w.cell_sizes)])
    nodes = np.concatenate([np.arange(starts[c], starts[c + 1]) for c in sorted(cells)])
    sub, keep = subset(w, nodes)
    sub.cell_sizes = np.asarray([w.cell_sizes[c] for c in sorted(cells)])  # type: ignore[attr-defined]
    return sub, keep
