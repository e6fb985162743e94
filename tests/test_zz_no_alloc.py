"""The allocation-free entry point mech_alloc_static (for callers that
cannot allocate device memory) against mech_alloc, through the C ABI: the
same workload gives the same bits on both contexts, on two calls in a row
with the second smaller; and the static area's limits."""
import numpy as np
import pytest

from paper_1905_02241_amd import mech, workloads as W
from tests.parity import compare_nodes, compare_states, log, run_oracle

pytestmark = pytest.mark.gpu


def _free_workload(seed, n_nodes):
    w = W.make_tiny(seed, kinds=("pas", "hh", "cahva", "syn"), n_nodes=n_nodes, per_node=2, syn_per_node=3.0,
                    vmode="isolated", event_rate_hz=300.0, nsteps=300)
    w.area[:] = np.linspace(100.0, 400.0, w.n_nodes)
    w.slots[-1].params["weight"][:] *= 6.0
    return w


def _run(w, static, path, nsteps=300):
    m = mech.from_workload(w, "fp64", static=static)
    if path == "resident":
        m.set_launch(128, 512, 256, 0, mech.LAUNCH_XCD_ORDER)
        m.set_resident_steps(64)
    m.step(nsteps, 0, w.dt, w.vmode, path)
    m.sync()
    return {"states": mech.states_of(m), **m.nodes(), "spikes": m.spike_counts()}, m


def _same(a, b, what):
    for key in ("v", "rhs", "d", "spikes"):
        assert np.array_equal(a[key], b[key]), (what, key)
    for s in range(len(a["states"])):
        for name, x in a["states"][s].items():
            assert np.array_equal(x, b["states"][s][name]), (what, s, name)


@pytest.mark.parametrize("path", ["batched", "resident"])
def test_static_context_equals_caller_buffer(path):
    """Two static contexts in a row, the second on a smaller workload, each
    against a context on a caller buffer (the fused paths' node sums are
    order-independent, so the bits agree) and against the oracle."""
    for seed, n_nodes in ((41, 1500), (42, 300)):
        w = _free_workload(seed, n_nodes)
        ref, mr = _run(w, False, path)
        got, ms = _run(w, True, path)
        assert ms.static and ms.buf is None
        _same(got, ref, (path, n_nodes))
        M = run_oracle(w, 300)
        assert np.array_equal(got["spikes"], M.spikes)
        compare_states(got, M, "fp64", label=f"static {path} {n_nodes}")
        compare_nodes({k: got[k] for k in ("v", "rhs", "d")}, M, "fp64", label=f"static {path} {n_nodes}")
        log(f"static {path} {n_nodes} nodes: {int(M.spikes.sum())} spikes, same bits as mech_alloc")
        ms.close()
        mr.close()


def test_static_area_limits():
    """One live static context per device; a context larger than the area
    is refused; the area is free again after mech_free."""
    w = _free_workload(43, 200)
    a = mech.from_workload(w, "fp64", static=True)
    with pytest.raises(mech.MechError) as e:
        mech.from_workload(w, "fp64", static=True)
    assert e.value.code == mech.ERR_STATE
    a.close()
    b = mech.from_workload(w, "fp64", static=True)
    big = np.arange(1 << 22, dtype=np.int32)
    with pytest.raises(mech.MechError) as e:
        mech.Mechanisms(1 << 22, [("hh", big)], static=True)
    assert e.value.code == mech.ERR_NOMEM
    b.step(10, 0, w.dt, w.vmode, "batched")
    b.sync()
    b.close()
