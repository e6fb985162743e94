"""ctypes binding of libmech.so (include/mech.h).

Argument marshalling only: every step of the mechanism path runs in the HIP
kernels of the library.  PyTorch provides device memory (one flat buffer for
the instance arrays, plus the node vectors) and the stream.  Importing this
module does not touch the GPU; loading the library does, and it raises if
``libmech.so`` has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmech.so")

OK, ERR_INVAL, ERR_RANGE, ERR_NOMEM, ERR_STATE, ERR_HIP, ERR_NONFINITE = 0, -1, -2, -3, -4, -5, -6
KIND = {"pas": 0, "hh": 1, "ih": 2, "cahva": 3, "syn": 4, "kmarkov": 5, "capump": 6, "cabuf": 7}
PREC = {"fp64": 0, "fp32": 1}
VMODE = {"external": 0, "clamp": 1, "isolated": 2, "cable": 3}
PATH = {"plain": 0, "batched": 1, "resident": 2}
GLOBAL_NAMES = ("celsius", "ena", "ek", "eh", "cao", "cai0", "tau_ca", "ca_gamma", "ca_depth", "e_syn",
                "mg", "tau_r_ampa", "tau_d_ampa", "tau_r_nmda", "tau_d_nmda", "event_rate_hz", "event_seed",
                "vthresh", "fd_dv", "analytic_conductance", "pade_cnexp", "pump_vmax", "pump_kp",
                "buf_total", "buf_kon", "buf_koff", "newton_iters", "shared_ca")

# Exported symbols of include/mech.h (checked by the CPU tests).
SYMBOLS = ("mech_required_bytes", "mech_alloc", "mech_alloc_static", "mech_bind_nodes", "mech_bind_clamp", "mech_cable_required_bytes",
           "mech_cable_plan",
           "mech_bind_cable", "mech_set_params",
           "mech_set_global", "mech_init", "mech_cur", "mech_state", "mech_step", "mech_set_launch",
           "mech_get_launch", "mech_set_resident_steps", "mech_autotune", "mech_autotune_resident", "mech_get_state", "mech_set_state", "mech_spike_counts",
           "mech_sync", "mech_info", "mech_probe_stream", "mech_last_error", "mech_strerror", "mech_free")
LAUNCH_XCD_ORDER = 1
LAUNCH_NONTEMPORAL = 2
LAUNCH_PLAIN_ATOMIC = 4


class MechError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mech error {code}: {msg}")
        self.code = code


class TypeDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("count", C.c_int64), ("node_index", C.POINTER(C.c_int32))]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmech.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1905_02241_amd.build` "
                          "(there is no CPU fallback)")
    try:
        import torch  # noqa: F401  -- loads the HIP runtime the library links against
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, dp, ip, lp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "mech_required_bytes": [C.c_int64, C.POINTER(TypeDesc), C.c_int, C.c_int, C.POINTER(C.c_size_t)],
        "mech_alloc": [C.POINTER(vp), C.c_int64, C.POINTER(TypeDesc), C.c_int, C.c_int, vp, C.c_size_t, vp],
        "mech_alloc_static": [C.POINTER(vp), C.c_int64, C.POINTER(TypeDesc), C.c_int, C.c_int, vp],
        "mech_bind_nodes": [vp, vp, vp, vp, vp, vp],
        "mech_bind_clamp": [vp, vp, vp, vp, vp],
        "mech_cable_required_bytes": [C.c_int64, ip, C.c_int32, C.POINTER(C.c_size_t)],
        "mech_cable_plan": [C.c_int64, ip, C.c_int32, ip, ip, C.c_int64],
        "mech_bind_cable": [vp, ip, vp, C.c_int32, vp, C.c_size_t],
        "mech_set_params": [vp, C.c_int, C.c_char_p, dp, C.c_int64],
        "mech_set_global": [vp, C.c_char_p, C.c_double],
        "mech_init": [vp],
        "mech_cur": [vp, C.c_int64, C.c_double, C.c_int],
        "mech_state": [vp, C.c_double],
        "mech_step": [vp, C.c_int64, C.c_int64, C.c_double, C.c_int, C.c_int],
        "mech_set_launch": [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int],
        "mech_get_launch": [vp, ip, ip, ip, ip, ip],
        "mech_set_resident_steps": [vp, C.c_int],
        "mech_autotune": [vp, C.c_double, C.c_int, C.c_int, C.c_int, dp],
        "mech_autotune_resident": [vp, C.c_double, C.c_int, C.c_int, C.c_int, dp],
        "mech_get_state": [vp, C.c_int, C.c_char_p, dp, C.c_int64],
        "mech_set_state": [vp, C.c_int, C.c_char_p, dp, C.c_int64],
        "mech_spike_counts": [vp, ip, C.c_int64],
        "mech_sync": [vp],
        "mech_info": [vp, lp, lp],
        "mech_probe_stream": [C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, C.c_size_t, vp],
        "mech_last_error": [vp],
        "mech_strerror": [C.c_int],
        "mech_free": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.mech_last_error.restype = C.c_char_p
    L.mech_strerror.restype = C.c_char_p
    L.mech_free.restype = None
    _lib = L
    return L


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Mechanisms:
    """One mechanism context on the current CUDA/HIP device.

    ``types`` is a list of (kind, node_index) pairs; node arrays are torch
    float64 tensors on the device owned by this object (``v``, ``rhs``,
    ``d``, ``area``, ``cm``, ``clamp``)."""

    def __init__(self, n_nodes: int, types, prec: str = "fp64", stream=None, device: str = "cuda",
                 static: bool = False):
        import torch
        self.torch = torch
        self.L = load_library()
        self.n_nodes = int(n_nodes)
        self.prec = prec
        self.kinds = [k for k, _ in types]
        self._nodeidx = [np.ascontiguousarray(ni, dtype=np.int32) for _, ni in types]
        self.counts = [int(a.shape[0]) for a in self._nodeidx]
        descs = (TypeDesc * max(1, len(types)))()
        for i, (k, _) in enumerate(types):
            descs[i].kind = KIND[k]
            descs[i].count = self.counts[i]
            descs[i].node_index = self._nodeidx[i].ctypes.data_as(C.POINTER(C.c_int32))
        self._descs = descs
        nbytes = C.c_size_t(0)
        self._check(self.L.mech_required_bytes(self.n_nodes, descs, len(types), PREC[prec], C.byref(nbytes)), None)
        self.nbytes = int(nbytes.value)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # torch's caching allocator returns 512-byte aligned blocks; a static
        # context takes the library's own device area instead (mech_alloc_static)
        self.static = bool(static)
        self.buf = None if self.static else torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.v = torch.full((self.n_nodes,), -65.0, **f64)
        self.rhs = torch.zeros(self.n_nodes, **f64)
        self.d = torch.zeros(self.n_nodes, **f64)
        self.area = torch.full((self.n_nodes,), 500.0, **f64)
        self.cm = torch.ones(self.n_nodes, **f64)
        self.clamp = [torch.zeros(self.n_nodes, **f64) for _ in range(4)]
        ctx = C.c_void_p()
        if self.static:
            self._check(self.L.mech_alloc_static(C.byref(ctx), self.n_nodes, descs, len(types), PREC[prec],
                                                 self.stream.cuda_stream), None)
        else:
            self._check(self.L.mech_alloc(C.byref(ctx), self.n_nodes, descs, len(types), PREC[prec],
                                          self.buf.data_ptr(), self.nbytes, self.stream.cuda_stream), None)
        self.ctx = ctx
        self._check(self.L.mech_bind_nodes(ctx, _ptr(self.v), _ptr(self.rhs), _ptr(self.d), _ptr(self.area),
                                           _ptr(self.cm)))
        self._check(self.L.mech_bind_clamp(ctx, *[_ptr(t) for t in self.clamp]))

    # ----------------------------------------------------------- helpers --
    def _check(self, rc: int, ctx="self"):
        if rc != OK:
            c = self.ctx if ctx == "self" else ctx
            msg = self.L.mech_last_error(c).decode()
            raise MechError(rc, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.L.mech_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- setup --
    def set_node_array(self, name: str, values):
        t = getattr(self, name)
        t.copy_(self.torch.as_tensor(np.asarray(values, dtype=np.float64)).to(self.device))

    def set_clamp(self, off, amp, freq, phase):
        for t, a in zip(self.clamp, (off, amp, freq, phase)):
            t.copy_(self.torch.as_tensor(np.asarray(a, dtype=np.float64)).to(self.device))

    def bind_cable(self, parent, g_axial, unit_nodes: int = 0):
        """Cell trees for the cable mode: parent (-1 at roots, Hines order,
        contiguous cells) and axial conductances in uS.  unit_nodes bounds
        the subtree one workgroup solves (0: the device's LDS capacity)."""
        par = np.ascontiguousarray(parent, dtype=np.int32)
        nbytes = C.c_size_t(0)
        ip = C.POINTER(C.c_int32)
        self._check(self.L.mech_cable_required_bytes(self.n_nodes, par.ctypes.data_as(ip), int(unit_nodes),
                                                     C.byref(nbytes)), None)
        self.cable_buf = self.torch.empty(max(int(nbytes.value), 256), dtype=self.torch.uint8, device=self.device)
        self.g_axial = self.torch.as_tensor(np.asarray(g_axial, dtype=np.float64)).to(self.device)
        self._check(self.L.mech_bind_cable(self.ctx, par.ctypes.data_as(ip), _ptr(self.g_axial), int(unit_nodes),
                                           self.cable_buf.data_ptr(), int(nbytes.value)))

    def set_params(self, slot: int, name: str, values):
        a = np.ascontiguousarray(np.atleast_1d(np.asarray(values, dtype=np.float64)))
        self._check(self.L.mech_set_params(self.ctx, slot, name.encode(), _dp(a), a.shape[0]))

    def set_global(self, name: str, value: float):
        self._check(self.L.mech_set_global(self.ctx, name.encode(), float(value)))

    def set_globals(self, g: Dict[str, float]):
        for k in GLOBAL_NAMES:
            if k in g:
                self.set_global(k, g[k])

    def init(self):
        self._check(self.L.mech_init(self.ctx))

    # -------------------------------------------------------------- step --
    def cur(self, k: int, dt: float, accumulate: bool = False):
        self._check(self.L.mech_cur(self.ctx, k, dt, int(accumulate)))

    def state(self, dt: float):
        self._check(self.L.mech_state(self.ctx, dt))

    def step(self, nsteps: int, k0: int, dt: float, vmode: str = "clamp", path: str = "batched"):
        self._check(self.L.mech_step(self.ctx, nsteps, k0, dt, VMODE[vmode], PATH[path]))

    def set_launch(self, block: int, tile_instances: int, tile_nodes: int, blocks_per_cu: int = 0,
                   flags: int = LAUNCH_XCD_ORDER):
        self._check(self.L.mech_set_launch(self.ctx, block, tile_instances, tile_nodes, blocks_per_cu, flags))

    def set_resident_steps(self, steps_per_launch: int):
        self._check(self.L.mech_set_resident_steps(self.ctx, steps_per_launch))

    def get_launch(self):
        v = [C.c_int32() for _ in range(5)]
        self._check(self.L.mech_get_launch(self.ctx, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def info(self):
        a, b = C.c_int64(), C.c_int64()
        self._check(self.L.mech_info(self.ctx, C.byref(a), C.byref(b)))
        return {"n_tiles": a.value, "max_tile_nodes": b.value}

    def autotune(self, dt: float, vmode: str, nsteps: int = 10, reps: int = 3, path: str = "batched") -> float:
        ms = C.c_double(0.0)
        fn = self.L.mech_autotune_resident if path == "resident" else self.L.mech_autotune
        self._check(fn(self.ctx, dt, VMODE[vmode], nsteps, reps, C.byref(ms)))
        return ms.value

    def sync(self):
        self._check(self.L.mech_sync(self.ctx))

    # ------------------------------------------------------------ output --
    def get_state(self, slot: int, name: str) -> np.ndarray:
        out = np.empty(self.counts[slot], dtype=np.float64)
        self._check(self.L.mech_get_state(self.ctx, slot, name.encode(), _dp(out), out.shape[0]))
        return out

    def set_state(self, slot: int, name: str, values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.L.mech_set_state(self.ctx, slot, name.encode(), _dp(a), a.shape[0]))

    def ion(self, name: str) -> np.ndarray:
        """Per-node calcium ion array, 'cai' (mM) or 'ica' (mA/cm2)."""
        out = np.empty(self.n_nodes, dtype=np.float64)
        self._check(self.L.mech_get_state(self.ctx, -1, name.encode(), _dp(out), self.n_nodes))
        return out

    def set_ion(self, name: str, values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.L.mech_set_state(self.ctx, -1, name.encode(), _dp(a), a.shape[0]))

    def spike_counts(self) -> np.ndarray:
        out = np.empty(self.n_nodes, dtype=np.int32)
        self._check(self.L.mech_spike_counts(self.ctx, out.ctypes.data_as(C.POINTER(C.c_int32)), self.n_nodes))
        return out

    def nodes(self) -> Dict[str, np.ndarray]:
        self.sync()
        return {k: getattr(self, k).cpu().numpy() for k in ("v", "rhs", "d")}


STATE_NAMES = {"pas": (), "hh": ("m", "h", "n"), "ih": ("m",), "cahva": ("m", "h", "cai"),
               "syn": ("A_ampa", "B_ampa", "A_nmda", "B_nmda"), "kmarkov": ("C1", "C2", "O"),
               "capump": ("m", "h", "cai"), "cabuf": ("m", "h", "cai", "cab")}
CA_KINDS = ("cahva", "capump", "cabuf")


PROBE_OPS = {"copy": 0, "read": 1, "write": 2, "triad": 3, "split": 4, "rmw7": 5, "rmw20": 6}
PROBE_FLAGS = {"nt_load": 1, "nt_store": 2, "8b": 4, "chunked": 8, "aosoa": 16, "tiled": 32}


def probe_stream(op: str = "copy", nbytes: int = 1 << 32, unroll: int = 4, blocks_per_cu: int = 8,
                 reps: int = 5, flags=()) -> float:
    """Achieved GB/s of the library's streaming probe over `nbytes` of HBM
    traffic (copy and split: nbytes/2 read + nbytes/2 written; triad:
    2 nbytes/3 read + nbytes/3 written; read, write: nbytes; rmw7: seven
    arrays of 7 nbytes/10 read, three of them rewritten; rmw20: twenty
    arrays of 20 nbytes/28 read, eight of them rewritten); median of `reps`
    launches timed with events on the current stream.  `flags` names
    MECH_PROBE_* options (nt_load, nt_store, 8b, chunked, aosoa, tiled).
    Checks every return code and, for the copy, the copied bytes."""
    import torch
    L = load_library()
    part = {"copy": 2, "split": 2, "triad": 3}.get(op, 1)
    fl = 0
    for f in flags:
        fl |= PROBE_FLAGS[f]
    if op == "rmw20":
        half = (nbytes * 20 // 28) // (160 * 2048) * (160 * 2048)
        src = torch.empty(16, dtype=torch.uint8, device="cuda")
        dst = torch.zeros(half // 8, dtype=torch.float64, device="cuda")
        dst.fill_(0.5)
    elif op == "rmw7":
        half = (nbytes * 7 // 10) // (56 * 256) * (56 * 256)
        src = torch.empty(16, dtype=torch.uint8, device="cuda")
        dst = torch.zeros(half // 8, dtype=torch.float64, device="cuda")
        dst.fill_(0.5)
    else:
        half = (nbytes // part) // 16 * 16
        src = torch.empty(2 * half if op == "triad" else half, dtype=torch.uint8, device="cuda")
        dst = torch.zeros(half if op != "read" else 256, dtype=torch.uint8, device="cuda")
        src.fill_(7)
    s = torch.cuda.current_stream()
    args = (PROBE_OPS[op], unroll, blocks_per_cu, fl, dst.data_ptr(), src.data_ptr(), half, s.cuda_stream)

    def launch():
        rc = L.mech_probe_stream(*args)
        if rc != OK:
            raise MechError(rc, L.mech_last_error(None).decode())

    launch()
    torch.cuda.synchronize()
    if op == "copy" and not bool((dst[:: 1 << 20] == 7).all()):
        raise RuntimeError("copy probe did not copy")
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        launch()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    ts.sort()
    moved = half * 10 // 7 if op == "rmw7" else half * 28 // 20 if op == "rmw20" else part * half
    del src, dst
    return moved / ts[len(ts) // 2] / 1e9


PLAN_ARRAYS = ("parent", "pos_node", "pos_par", "pos_src", "elim_n", "elim_p", "elim_ptr", "unit_pos",
               "unit_elim", "unit_mode", "list_up", "list_top", "list_top_g", "list_down")


def cable_plan(parent, unit_nodes: int = 0) -> Dict[str, np.ndarray]:
    """The cut of the cell trees that bind_cable makes (mech_cable_plan),
    as host arrays by name; host only."""
    L = load_library()
    par = np.ascontiguousarray(parent, dtype=np.int32)
    ip = C.POINTER(C.c_int32)
    sizes = np.zeros(len(PLAN_ARRAYS), dtype=np.int32)
    rc = L.mech_cable_plan(par.shape[0], par.ctypes.data_as(ip), int(unit_nodes), sizes.ctypes.data_as(ip), None, 0)
    if rc != OK:
        raise MechError(rc, L.mech_last_error(None).decode())
    buf = np.zeros(max(int(sizes.sum()), 1), dtype=np.int32)
    rc = L.mech_cable_plan(par.shape[0], par.ctypes.data_as(ip), int(unit_nodes), sizes.ctypes.data_as(ip),
                           buf.ctypes.data_as(ip), buf.shape[0])
    if rc != OK:
        raise MechError(rc, L.mech_last_error(None).decode())
    out, k = {}, 0
    for name, n in zip(PLAN_ARRAYS, sizes):
        out[name] = buf[k:k + n].copy()
        k += n
    return out


def from_workload(w, prec: str = "fp64", init: bool = True, unit_nodes: int = 0, static: bool = False) -> Mechanisms:
    """Build a context from a workload (paper_1905_02241_amd.workloads):
    node index, parameters, globals, node arrays (and cell trees, cut into
    units of at most unit_nodes, 0 for the device's capacity); v = v_init
    everywhere and, if `init`, every STATE at its steady state there.
    static: the context lives in the library's static device area
    (mech_alloc_static)."""
    m = Mechanisms(w.n_nodes, [(s.kind, s.node) for s in w.slots], prec=prec, static=static)
    m.set_globals(w.globals)
    for i, s in enumerate(w.slots):
        for name, vals in s.params.items():
            m.set_params(i, name, vals)
    if w.area is not None:
        m.set_node_array("area", w.area)
    if w.cm is not None:
        m.set_node_array("cm", w.cm)
    if w.clamp_off is not None:
        m.set_clamp(w.clamp_off, w.clamp_amp, w.clamp_freq, w.clamp_phase)
    if getattr(w, "parent", None) is not None:
        m.bind_cable(w.parent, w.g_axial, unit_nodes)
    m.v.fill_(float(w.v_init))
    if init:
        m.init()
    return m


def states_of(m: Mechanisms) -> List[Dict[str, np.ndarray]]:
    out = []
    for i, k in enumerate(m.kinds):
        d = {name: m.get_state(i, name) for name in STATE_NAMES[k]}
        if k in CA_KINDS:
            d["ica"] = m.get_state(i, "ica")
        out.append(d)
    return out
