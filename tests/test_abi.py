"""CPU checks of the C ABI: the library loads, exports every function that
include/mech.h declares, and its host-side validation (which runs before any
device call) rejects bad input with the documented codes."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1905_02241_amd import mech

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mech.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mech_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mech.LIB_PATH):
        from paper_1905_02241_amd import build
        build.build()
    return mech.load_library()


def test_header_declares_the_binding_symbols():
    assert declared_functions() == sorted(mech.SYMBOLS)


def declared_arity():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(mech_[a-z_]+)\s*\(([^)]*)\)\s*;", src):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argtypes_match_header_arity(lib):
    for name, n in declared_arity().items():
        assert len(getattr(lib, name).argtypes) == n, name


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_codes(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.mech_strerror(code)
    assert lib.mech_strerror(0) == b"ok"
    assert lib.mech_strerror(-2) == b"node index out of range"


def _descs(types):
    d = (mech.TypeDesc * max(1, len(types)))()
    keep = []
    for i, (k, ni) in enumerate(types):
        a = np.ascontiguousarray(ni, dtype=np.int32)
        keep.append(a)
        d[i].kind = mech.KIND[k] if isinstance(k, str) else k
        d[i].count = a.shape[0]
        d[i].node_index = a.ctypes.data_as(C.POINTER(C.c_int32))
    return d, keep


def test_required_bytes_layout(lib):
    out = C.c_size_t()
    d, keep = _descs([("hh", np.arange(1000))])
    assert lib.mech_required_bytes(1000, d, 1, 0, C.byref(out)) == 0
    fp64 = out.value
    assert lib.mech_required_bytes(1000, d, 1, 1, C.byref(out)) == 0
    fp32 = out.value
    # 1024 padded instances: index 4 B, 3 states and 4 parameters (the three
    # conductances and el) in the state type
    inst64 = 1024 * (4 + 3 * 8 + 4 * 8)
    inst32 = 1024 * (4 + 3 * 4 + 4 * 4)
    assert fp64 - fp32 == inst64 - inst32
    assert fp64 % 256 == 0 and fp64 > inst64


def test_required_bytes_cabuf_layout(lib):
    """The buffered-calcium type: index, four STATEs (m, h, cai, cab), gbar
    and its calcium current per padded instance, and the per-node ion region
    (cai, ica) that every calcium type brings."""
    out = C.c_size_t()
    d, keep = _descs([("cabuf", np.arange(1000))])
    assert lib.mech_required_bytes(1000, d, 1, 0, C.byref(out)) == 0
    fp64 = out.value
    assert lib.mech_required_bytes(1000, d, 1, 1, C.byref(out)) == 0
    fp32 = out.value
    inst64 = 1024 * (4 + 4 * 8 + 8 + 8)
    inst32 = 1024 * (4 + 4 * 4 + 4 + 4)
    assert fp64 - fp32 == inst64 - inst32
    assert fp64 > inst64 + 16 * 1000
    d, keep = _descs([(8, np.arange(4))])
    assert lib.mech_required_bytes(4, d, 1, 0, C.byref(out)) == mech.ERR_INVAL


def test_validation_codes(lib):
    out = C.c_size_t()
    d, keep = _descs([(9, np.arange(4))])
    assert lib.mech_required_bytes(4, d, 1, 0, C.byref(out)) == mech.ERR_INVAL
    d, keep = _descs([("hh", np.arange(4))])
    assert lib.mech_required_bytes(4, d, 1, 7, C.byref(out)) == mech.ERR_INVAL
    assert lib.mech_required_bytes(-1, d, 1, 0, C.byref(out)) == mech.ERR_INVAL
    assert lib.mech_required_bytes(4, d, 9, 0, C.byref(out)) == mech.ERR_INVAL
    # mech_alloc rejects on the host, before any device call: a fake aligned
    # buffer address is never dereferenced on these paths
    ctx = C.c_void_p()
    fake = 1 << 20
    d, keep = _descs([("hh", np.array([0, 1, 4]))])
    assert lib.mech_alloc(C.byref(ctx), 4, d, 1, 0, fake, 1 << 30, None) == mech.ERR_RANGE
    assert b"outside" in lib.mech_last_error(None)
    d, keep = _descs([("hh", np.array([0, 1, -1]))])
    assert lib.mech_alloc(C.byref(ctx), 4, d, 1, 0, fake, 1 << 30, None) == mech.ERR_RANGE
    d, keep = _descs([("hh", np.array([0, 1, 2]))])
    assert lib.mech_alloc(C.byref(ctx), 4, d, 1, 0, fake, 16, None) == mech.ERR_NOMEM
    assert lib.mech_alloc(C.byref(ctx), 4, d, 1, 0, fake + 8, 1 << 30, None) == mech.ERR_INVAL
    assert lib.mech_alloc(C.byref(ctx), 4, d, 1, 0, None, 1 << 30, None) == mech.ERR_INVAL
    # at most 2^19 instances on one node, all types together (the bound of
    # the fused paths' fixed-point node sums)
    d, keep = _descs([("syn", np.zeros((1 << 19) - 1, dtype=np.int32)), ("pas", np.arange(4))])
    assert lib.mech_alloc(C.byref(ctx), 4, d, 2, 0, fake, 16, None) == mech.ERR_NOMEM
    d, keep = _descs([("syn", np.zeros(1 << 19, dtype=np.int32)), ("pas", np.arange(4))])
    assert lib.mech_alloc(C.byref(ctx), 4, d, 2, 0, fake, 1 << 30, None) == mech.ERR_INVAL
    assert b"more than" in lib.mech_last_error(None)
    # the static area (mech_alloc_static) rejects contexts larger than it
    # before any device call
    d, keep = _descs([("hh", np.arange(1 << 22, dtype=np.int32))])
    assert lib.mech_alloc_static(C.byref(ctx), 1 << 22, d, 1, 0, None) == mech.ERR_NOMEM
    assert b"static area" in lib.mech_last_error(None)
    d, keep = _descs([(9, np.arange(4))])
    assert lib.mech_alloc_static(C.byref(ctx), 4, d, 1, 0, None) == mech.ERR_INVAL
    assert lib.mech_alloc_static(None, 4, d, 1, 0, None) == mech.ERR_INVAL
    assert not ctx.value
    # null-context calls
    assert lib.mech_init(None) == mech.ERR_INVAL
    assert lib.mech_step(None, 1, 0, 0.025, 1, 1) == mech.ERR_INVAL
    assert lib.mech_sync(None) == mech.ERR_INVAL
    lib.mech_free(None)


def test_staged_kind_shapes_match_the_kind_tables(lib, tmp_path):
    """The time-fused kernels stage each kind by a compile-time shape
    (mech_internal.h).  It must match the binding's variable tables and the
    library's buffer layout (mech_required_bytes in both precisions)."""
    from paper_1905_02241_amd import workloads as W
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_1905_02241_amd", "csrc")
    exe = str(tmp_path / "kind_shapes")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                        os.path.join(ROOT, "tests", "kind_shapes.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    shapes = {int(f[0]): tuple(int(x) for x in f[1:]) for f in (l.split() for l in out if l.strip())}
    assert sorted(shapes) == list(range(len(W.KINDS)))
    for kind, kid in mech.KIND.items():
        n_state, n_param, dbl, ica, gid = shapes[kid]
        assert n_state == len(mech.STATE_NAMES[kind]), kind
        assert n_param == len(W.PARAM_NAMES[kind]), kind
        assert ica == (kind in mech.CA_KINDS), kind
        assert gid == (kind == "syn"), kind
        # bytes per 64 padded instances in each precision, from the library
        d, keep = _descs([(kind, np.arange(64))])
        out64, out32 = C.c_size_t(), C.c_size_t()
        assert lib.mech_required_bytes(64, d, 1, 0, C.byref(out64)) == 0
        assert lib.mech_required_bytes(64, d, 1, 1, C.byref(out32)) == 0
        n_dbl = bin(dbl).count("1")
        per8 = n_state + n_param + ica          # 8-byte values per instance in FP64
        per4 = n_state + (n_param - n_dbl) + ica  # values that shrink to 4 bytes in FP32
        assert out64.value - out32.value == 64 * 4 * per4, (kind, per8, per4)
