"""ctypes binding of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
module.  It loads ``liboracle.so`` built from ``mech_oracle.c`` by plain gcc
with -O2 -fno-fast-math -ffp-contract=off (``build()``), and it imports
nothing from the GPU package: a workload is read through its attributes
(``n_nodes``, ``slots[i].kind/.node/.params/.gid``, ``area``, ``cm``,
``clamp_*``, ``globals``, ``vmode``, ``dt``, ``v_init``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, List

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mech_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

KIND = {"pas": 0, "hh": 1, "ih": 2, "cahva": 3, "syn": 4, "kmarkov": 5, "capump": 6, "cabuf": 7}
VMODE = {"external": 0, "clamp": 1, "isolated": 2, "cable": 3}
PARAMS = {"pas": ("g", "e"), "hh": ("gnabar", "gkbar", "gl", "el"), "ih": ("gbar",),
          "cahva": ("gbar",), "syn": ("weight",), "kmarkov": ("gbar",), "capump": ("gbar",), "cabuf": ("gbar",)}
STATES = {"pas": (), "hh": ("m", "h", "n"), "ih": ("m",), "cahva": ("m", "h", "cai"),
          "syn": ("A_ampa", "B_ampa", "A_nmda", "B_nmda"), "kmarkov": ("C1", "C2", "O"),
          "capump": ("m", "h", "cai"), "cabuf": ("m", "h", "cai", "cab")}
GLOBAL_FIELDS = ("celsius", "ena", "ek", "eh", "cao", "cai0", "tau_ca", "ca_gamma", "ca_depth",
                 "e_syn", "mg", "tau_r_ampa", "tau_d_ampa", "tau_r_nmda", "tau_d_nmda",
                 "event_rate_hz", "vthresh", "fd_dv")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class _Slot(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("node", _ip), ("gid", _lp),
                ("st", _dp * 4), ("par", _dp * 4), ("ica", _dp)]


FLAG_FIELDS = ("analytic_conductance", "pade_cnexp")


class _Globals(C.Structure):
    _fields_ = ([(f, C.c_double) for f in GLOBAL_FIELDS] + [("event_seed", C.c_uint64)] +
                [(f, C.c_int32) for f in FLAG_FIELDS] +
                [("pump_vmax", C.c_double), ("pump_kp", C.c_double), ("newton_iters", C.c_int32),
                 ("shared_ca", C.c_int32), ("buf_total", C.c_double), ("buf_kon", C.c_double),
                 ("buf_koff", C.c_double)])


class _Nodes(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("v", _dp), ("rhs", _dp), ("d", _dp), ("area", _dp), ("cm", _dp),
                ("clamp_off", _dp), ("clamp_amp", _dp), ("clamp_freq", _dp), ("clamp_phase", _dp),
                ("spikes", _ip), ("parent", _ip), ("g_axial", _dp), ("cai", _dp), ("ica", _dp)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99, strict IEEE, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "mech_oracle.h"))):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_hh_inf_tau.argtypes = [C.c_double, C.c_double, _dp]
        L.orc_hh_rates.argtypes = [C.c_double, _dp]
        L.orc_ih_inf_tau.argtypes = [C.c_double, _dp]
        L.orc_cahva_inf_tau.argtypes = [C.c_double, _dp]
        L.orc_mg_block.argtypes = [C.c_double, C.c_double]
        L.orc_mg_block.restype = C.c_double
        L.orc_syn_peak_factor.argtypes = [C.c_double, C.c_double, _dp]
        L.orc_syn_peak_factor.restype = C.c_double
        L.orc_nernst_ca.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_nernst_ca.restype = C.c_double
        L.orc_ca_kappa.argtypes = [C.c_double, C.c_double]
        L.orc_ca_kappa.restype = C.c_double
        L.orc_event_hash.argtypes = [C.c_uint64, C.c_int64, C.c_int64]
        L.orc_event_hash.restype = C.c_uint64
        L.orc_event_threshold.argtypes = [C.c_double, C.c_double]
        L.orc_event_threshold.restype = C.c_uint64
        L.orc_kmarkov_matrix.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        L.orc_kmarkov_step.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        L.orc_capump_step.argtypes = [C.POINTER(_Globals), C.c_double, C.c_double, _dp, C.c_int]
        L.orc_capump_step.restype = C.c_double
        L.orc_cabuf_step.argtypes = [C.POINTER(_Globals), C.c_double, C.c_double, _dp, _dp, C.c_int]
        L.orc_cabuf_step.restype = C.c_double
        L.orc_cabuf_bound.argtypes = [C.POINTER(_Globals), C.c_double]
        L.orc_cabuf_bound.restype = C.c_double
        L.orc_instance_current.argtypes = [C.POINTER(_Globals), C.POINTER(_Nodes), C.POINTER(_Slot), C.c_int64,
                                           C.c_double, _dp, _dp]
        L.orc_node_scales.argtypes = [C.POINTER(_Globals), C.POINTER(_Nodes), C.POINTER(_Slot), C.c_int, _dp, _dp,
                                      _ip]
        sig = [C.POINTER(_Globals), C.POINTER(_Nodes), C.POINTER(_Slot), C.c_int]
        L.orc_init.argtypes = sig
        L.orc_cur.argtypes = sig
        L.orc_events.argtypes = [C.POINTER(_Globals), C.POINTER(_Slot), C.c_int, C.c_int64, C.c_double]
        L.orc_vclamp.argtypes = [C.POINTER(_Nodes), C.c_double]
        L.orc_visolated.argtypes = [C.POINTER(_Globals), C.POINTER(_Nodes), C.c_double]
        L.orc_vcable.argtypes = [C.POINTER(_Globals), C.POINTER(_Nodes), C.c_double]
        L.orc_state.argtypes = sig + [C.c_double]
        L.orc_run.argtypes = sig + [C.c_int64, C.c_int64, C.c_double, C.c_int]
        L.orc_run.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


# ------------------------------------------------------------ scalar API --
def hh_inf_tau(v: float, celsius: float = 6.3) -> np.ndarray:
    o = np.zeros(6)
    lib().orc_hh_inf_tau(v, celsius, _ptr(o))
    return o


def hh_rates(v: float) -> np.ndarray:
    o = np.zeros(6)
    lib().orc_hh_rates(v, _ptr(o))
    return o


def ih_inf_tau(v: float) -> np.ndarray:
    o = np.zeros(2)
    lib().orc_ih_inf_tau(v, _ptr(o))
    return o


def cahva_inf_tau(v: float) -> np.ndarray:
    o = np.zeros(4)
    lib().orc_cahva_inf_tau(v, _ptr(o))
    return o


def mg_block(v: float, mg: float = 1.0) -> float:
    return lib().orc_mg_block(v, mg)


def syn_peak_factor(tau_r: float, tau_d: float):
    tp = C.c_double(0.0)
    f = lib().orc_syn_peak_factor(tau_r, tau_d, C.byref(tp))
    return f, tp.value


def nernst_ca(cai: float, cao: float, celsius: float) -> float:
    return lib().orc_nernst_ca(cai, cao, celsius)


def ca_kappa(gamma: float, depth: float) -> float:
    return lib().orc_ca_kappa(gamma, depth)


def event_hash(seed: int, gid: int, k: int) -> int:
    return int(lib().orc_event_hash(seed, gid, k))


def event_threshold(rate_hz: float, dt: float) -> int:
    return int(lib().orc_event_threshold(rate_hz, dt))


def kmarkov_matrix(v: float, celsius: float, dt: float) -> np.ndarray:
    M = np.zeros(9)
    lib().orc_kmarkov_matrix(v, celsius, dt, _ptr(M))
    return M.reshape(3, 3)


def kmarkov_step(v: float, celsius: float, dt: float, x) -> np.ndarray:
    x = np.array(x, dtype=np.float64)
    lib().orc_kmarkov_step(v, celsius, dt, _ptr(x))
    return x


# ----------------------------------------------------------------- model --
class Model:
    """Owns FP64 copies of one workload's arrays and runs the oracle on them.

    ``states[s][name]`` are the STATE arrays of slot s in the caller's
    instance order, ``ica[s]`` the calcium current of each instance of a
    calcium slot; ``v``, ``rhs``, ``d``, ``spikes`` and, under shared_ca,
    ``cai_node`` and ``ica_node`` are node arrays."""

    def __init__(self, w):
        self.w = w
        self.n_nodes = int(w.n_nodes)
        n = self.n_nodes
        self.v = np.full(n, float(w.v_init))
        self.rhs = np.zeros(n)
        self.d = np.zeros(n)
        self.spikes = np.zeros(n, dtype=np.int32)
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        self.area, self.cm = f64(w.area), f64(w.cm)
        self.clamp = [f64(getattr(w, "clamp_" + k)) for k in ("off", "amp", "freq", "phase")]
        self.globals = dict(w.globals)
        self.dt = float(w.dt)
        self.vmode = w.vmode
        self.states: List[Dict[str, np.ndarray]] = []
        self.ica: List[np.ndarray] = []
        self._keep = []
        self._slots = (_Slot * max(1, len(w.slots)))()
        for i, s in enumerate(w.slots):
            node = np.ascontiguousarray(s.node, dtype=np.int32)
            if node.size and (node.min() < 0 or node.max() >= n):
                raise ValueError("node index out of range")
            gid = None if s.gid is None else np.ascontiguousarray(s.gid, dtype=np.int64)
            st = {name: np.zeros(node.shape[0]) for name in STATES[s.kind]}
            par = [np.ascontiguousarray(s.params[p], dtype=np.float64) for p in PARAMS[s.kind]]
            ica = np.zeros(node.shape[0])
            self.states.append(st)
            self.ica.append(ica)
            self._keep.append((node, gid, par))
            sl = self._slots[i]
            sl.kind = KIND[s.kind]
            sl.n = node.shape[0]
            sl.node = _ptr(node, _ip)
            sl.gid = _ptr(gid, _lp) if gid is not None else None
            for j, name in enumerate(STATES[s.kind]):
                sl.st[j] = _ptr(st[name])
            for j, a in enumerate(par):
                sl.par[j] = _ptr(a)
            sl.ica = _ptr(ica)
        self.nslots = len(w.slots)
        par = getattr(w, "parent", None)
        self.parent = None if par is None else np.ascontiguousarray(par, dtype=np.int32)
        self.g_axial = f64(getattr(w, "g_axial", None))
        if self.parent is not None and self.parent.size and np.any(self.parent >= np.arange(n)):
            raise ValueError("parent[n] must be < n (Hines order)")
        # per-node calcium (shared_ca): concentration and total current
        self.cai_node = np.full(n, float(self.globals["cai0"]))
        self.ica_node = np.zeros(n)
        self._nodes = _Nodes(n, _ptr(self.v), _ptr(self.rhs), _ptr(self.d), _ptr(self.area), _ptr(self.cm),
                             *[_ptr(a) for a in self.clamp], _ptr(self.spikes, _ip),
                             _ptr(self.parent, _ip), _ptr(self.g_axial), _ptr(self.cai_node),
                             _ptr(self.ica_node))
        self._g = self._make_globals()

    def _make_globals(self):
        g = _Globals()
        for f in GLOBAL_FIELDS:
            setattr(g, f, float(self.globals[f]))
        g.event_seed = int(self.globals["event_seed"]) & ((1 << 64) - 1)
        for f in FLAG_FIELDS:
            setattr(g, f, int(self.globals.get(f, 0)))
        g.pump_vmax = float(self.globals.get("pump_vmax", 1e-4))
        g.pump_kp = float(self.globals.get("pump_kp", 1e-3))
        g.newton_iters = int(self.globals.get("newton_iters", 4))
        g.shared_ca = int(self.globals.get("shared_ca", 0))
        g.buf_total = float(self.globals.get("buf_total", 0.05))
        g.buf_kon = float(self.globals.get("buf_kon", 100.0))
        g.buf_koff = float(self.globals.get("buf_koff", 0.1))
        return g

    def set_global(self, name, value):
        self.globals[name] = value
        self._g = self._make_globals()

    def _args(self):
        return C.byref(self._g), C.byref(self._nodes), self._slots, self.nslots

    def init(self, v_init=None):
        """v = v_init everywhere, then every STATE at its steady state."""
        self.v[:] = self.w.v_init if v_init is None else v_init
        lib().orc_init(*self._args())

    def events(self, k: int):
        lib().orc_events(C.byref(self._g), self._slots, self.nslots, k, self.dt)

    def cur(self):
        lib().orc_cur(*self._args())

    def state(self):
        lib().orc_state(*self._args(), self.dt)

    def vclamp(self, t: float):
        lib().orc_vclamp(C.byref(self._nodes), t)

    def visolated(self):
        lib().orc_visolated(C.byref(self._g), C.byref(self._nodes), self.dt)

    def vcable(self):
        lib().orc_vcable(C.byref(self._g), C.byref(self._nodes), self.dt)

    def run(self, k0: int, nsteps: int, vmode=None):
        vm = VMODE[vmode or self.vmode]
        if vm == 1 and any(a is None for a in self.clamp):
            raise ValueError("clamp mode needs clamp arrays")
        if vm in (2, 3) and self.cm is None:
            raise ValueError("isolated and cable modes need cm")
        if vm == 3 and (self.parent is None or self.g_axial is None or self.area is None):
            raise ValueError("cable mode needs parent, g_axial and area")
        r = lib().orc_run(*self._args(), k0, nsteps, self.dt, vm)
        if r != 0:
            raise ValueError("orc_run rejected its arguments")

    def capump_step(self, ica: float, cai: float, iters: int):
        """One implicit Euler step of the capump pool; returns (cai, residual)."""
        c = C.c_double(cai)
        r = lib().orc_capump_step(C.byref(self._g), ica, self.dt, C.byref(c), iters)
        return c.value, r

    def cabuf_step(self, ica: float, cai: float, cab: float, iters: int, dt=None):
        """One implicit Euler step of the cabuf pool; returns (cai, cab, residual)."""
        c, b = C.c_double(cai), C.c_double(cab)
        r = lib().orc_cabuf_step(C.byref(self._g), ica, self.dt if dt is None else dt, C.byref(c), C.byref(b), iters)
        return c.value, b.value, r

    def cabuf_bound(self, cai: float) -> float:
        return lib().orc_cabuf_bound(C.byref(self._g), cai)

    def node_scales(self):
        """Rounding scales of the current update at the model's v and STATEs
        (orc_node_scales): per node the summed term magnitudes |s| T_i, the
        summed |s g_i| and the number of instances.  For tolerances only."""
        n = self.n_nodes
        terms, gsum, cnt = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int32)
        lib().orc_node_scales(C.byref(self._g), C.byref(self._nodes), self._slots, self.nslots, _ptr(terms),
                              _ptr(gsum), _ptr(cnt, _ip))
        return terms, gsum, cnt

    def instance_current(self, s: int, i: int, v: float):
        cur, cond = C.c_double(), C.c_double()
        lib().orc_instance_current(C.byref(self._g), C.byref(self._nodes), C.byref(self._slots[s]), i, v,
                                   C.byref(cur), C.byref(cond))
        return cur.value, cond.value
