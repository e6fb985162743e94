"""The sharded oracle run used for large node samples: nodes cut into ranges,
each range run by the single-threaded oracle in its own thread, results
merged.  Nodes are independent under a clamp and in isolated mode, so the
merged run must equal one single-threaded run bit for bit."""
import numpy as np
import pytest

from paper_1905_02241_amd import workloads as W
from tests.parity import run_oracle, run_oracle_sharded


@pytest.mark.parametrize("vmode", ["clamp", "isolated"])
@pytest.mark.parametrize("parts", [1, 3, 8])
def test_sharded_oracle_equals_single_run(vmode, parts):
    w = W.make_tiny(5, kinds=("pas", "hh", "ih", "cahva", "syn"), n_nodes=120, per_node=2, vmode=vmode,
                    event_rate_hz=300.0, nsteps=200)
    w.slots[-1].params["weight"][:] *= 6.0
    a = run_oracle(w, 200)
    b = run_oracle_sharded(w, 200, parts=parts)
    for key in ("v", "rhs", "d", "spikes"):
        assert np.array_equal(getattr(a, key), getattr(b, key)), key
    for s in range(len(w.slots)):
        for name in a.states[s]:
            assert np.array_equal(a.states[s][name], b.states[s][name]), (s, name)
        assert np.array_equal(a.ica[s], b.ica[s]), s


def test_sharded_oracle_shared_calcium():
    w = W.make_tiny(6, kinds=("pas", "hh", "cahva", "capump", "syn"), n_nodes=90, per_node=2, vmode="isolated",
                    nsteps=150)
    w.globals["shared_ca"] = 1
    a = run_oracle(w, 150)
    b = run_oracle_sharded(w, 150, parts=4)
    for key in ("v", "cai_node", "ica_node"):
        assert np.array_equal(getattr(a, key), getattr(b, key)), key


def test_sharded_oracle_rejects_cable():
    w = W.make_tiny(7, n_nodes=20, vmode="isolated")
    w.vmode = "cable"
    with pytest.raises(ValueError):
        run_oracle_sharded(w, 10)
