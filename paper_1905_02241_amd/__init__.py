"""MI355X mechanism kernels: nrn_cur / nrn_state of NMODL-style membrane
mechanisms as hand-written HIP kernels for gfx950 behind the C ABI of
include/mech.h.  ``mech`` is the ctypes binding, ``workloads`` the seeded
synthetic inputs, ``build`` compiles libmech.so in-tree."""
__all__ = ["mech", "workloads", "build"]
