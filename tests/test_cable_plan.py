"""CPU checks of the host-side cut of cell trees for the cable mode
(mech_cable_plan): structural invariants of the plan, and a replay of its
schedule with the kernels' semantics (all records of one height read their
operands before any of them writes, units of one launch are independent)
whose voltage step must equal the oracle's Hines solve (backward Euler of
the cable equation, section 5.2's "Other" phase of a step) up to rounding.
A schedule that reads a row before it is final, drops an edge, or hands a
wrong row between the passes changes dv by O(1)."""
import types

import numpy as np
import pytest

from paper_1905_02241_amd import mech, workloads as W

FULL, PIECE, TOP = 0, 1, 2


def cells(seed, sizes, mean_section=8.0):
    rng = np.random.default_rng(seed)
    parts, first = [], 0
    for sz in sizes:
        parts.append(W.random_cell(rng, int(sz), first, mean_section))
        first += int(sz)
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(3))


def chain(n, first=0):
    par = np.arange(first - 1, first + n - 1, dtype=np.int32)
    par[0] = -1
    return par


def star(n, first=0):
    par = np.full(n, first, dtype=np.int32)
    par[0] = -1
    return par


def geometry(rng, parent):
    n = parent.shape[0]
    area = rng.uniform(50.0, 800.0, n)
    g = rng.uniform(0.01, 0.5, n)
    g[parent < 0] = 0.0
    return area, g


def check_structure(plan, n, cap):
    pn, pp, ps = plan["pos_node"], plan["pos_par"], plan["pos_src"]
    up, ue, um = plan["unit_pos"], plan["unit_elim"], plan["unit_mode"]
    par = plan["parent"]
    U = um.shape[0]
    assert up[0] == 0 and up[-1] == pn.shape[0] and np.all(np.diff(up) >= 1)
    unit_of = np.repeat(np.arange(U), np.diff(up))
    # every node has exactly one own position; ghosts repeat piece roots
    own = ps < 0
    assert np.array_equal(np.sort(pn[own]), np.arange(n))
    g = np.flatnonzero(~own)
    assert np.all(pn[ps[g]] == pn[g]) and np.all(um[unit_of[ps[g]]] == PIECE)
    assert np.all(um[unit_of[g]] == TOP) and np.all(pp[ps[g]] == -1)
    # a parent row in the same unit, of the node's parent
    has = pp >= 0
    assert np.all(unit_of[pp[has]] == unit_of[has]) and np.all(pn[pp[has]] == par[pn[has]])
    assert np.all((par[pn[~has]] < 0) | (um[unit_of[~has]] == PIECE))
    # one record per node: an edge, or a root's own record
    assert plan["elim_n"].shape[0] == n
    # sizes and launch lists
    size = np.diff(up)
    assert np.all(size[um != TOP] <= cap)
    assert sorted(plan["list_up"].tolist()) == np.flatnonzero(um != TOP).tolist()
    assert sorted(plan["list_down"].tolist()) == np.flatnonzero(um != TOP).tolist()
    tops = sorted(plan["list_top"].tolist() + plan["list_top_g"].tolist())
    assert tops == np.flatnonzero(um == TOP).tolist()
    assert np.all(size[plan["list_top"]] <= cap) and np.all(size[plan["list_top_g"]] > cap)
    assert ue[0] == 0 and ue[-1] == plan["elim_ptr"].shape[0] - 1


def replay(plan, v, rhs, d, cm, area, g, dt):
    """The unit schedule on the CPU, with the kernels' per-height semantics."""
    par, pn, ps = plan["parent"], plan["pos_node"], plan["pos_src"]
    en, ep, eptr = plan["elim_n"], plan["elim_p"], plan["elim_ptr"]
    up, ue, um = plan["unit_pos"], plan["unit_elim"], plan["unit_mode"]
    has = par >= 0
    pa = np.where(has, par, 0)
    kn = np.where(has, 1e2 * g / area, 0.0)
    kp = np.where(has, 1e2 * g / area[pa], 0.0)
    rnode = pn[en]
    ekn, ekp = kn[rnode], kp[rnode]
    P = pn.shape[0]
    GD, GR = np.zeros(P), np.zeros(P)
    vout = v.copy()

    def unit(u, down):
        p0, p1 = up[u], up[u + 1]
        L0, L1 = ue[u], ue[u + 1]
        nlev = L1 - L0
        D, R = np.zeros(P), np.zeros(P)
        idx = np.arange(p0, p1)
        if not down:
            n = pn[idx]
            dv = np.where(has[n], v[pa[n]] - v[n], 0.0)
            ghost = ps[idx] >= 0
            Dn = np.where(ghost, GD[np.maximum(ps[idx], 0)], 1e-3 * cm[n] / dt + d[n] + kn[n])
            Rn = np.where(ghost, GR[np.maximum(ps[idx], 0)], rhs[n] + kn[n] * dv)
            # every position writes its own row; a child's coupling terms go
            # to its parent with its fold
            D[idx], R[idx] = Dn, Rn
            DV = np.zeros(P)
            DV[idx] = dv
            nel = nlev if um[u] == PIECE else nlev - 1
            for j in range(nel):
                q = np.arange(eptr[L0 + j], eptr[L0 + j + 1])
                rn, rp = en[q], ep[q]
                assert np.all(rn != rp)
                # a height's records sorted by parent: one thread folds each run
                assert np.all(np.diff(rp) >= 0)
                Dc, Rc = D[rn].copy(), R[rn].copy()
                f = ekp[q] / Dc
                np.add.at(D, rp, ekp[q] - f * ekn[q])
                np.add.at(R, rp, f * Rc - ekp[q] * DV[rn])
            if um[u] != TOP:
                # whole cells and pieces back-substitute in the second pass
                GD[idx], GR[idx] = D[idx], R[idx]
                return
        else:
            D[idx], R[idx] = GD[idx], GR[idx]
        for j in range(nlev - 1, -1, -1):
            q = np.arange(eptr[L0 + j], eptr[L0 + j + 1])
            rn, rp = en[q], ep[q]
            Rp = R[rp].copy()
            R[rn] = (R[rn] + ekn[q] * Rp) / D[rn]
        for i in idx:
            if ps[i] >= 0:
                GR[ps[i]] = R[i]
            else:
                vout[pn[i]] += R[i]

    for u in plan["list_up"]:
        unit(u, False)
    for u in np.concatenate([plan["list_top"], plan["list_top_g"]]):
        unit(u, False)
    for u in plan["list_down"]:
        unit(u, True)
    return vout


def oracle_step(oracle, parent, area, g, v, rhs, d, cm, dt):
    n = parent.shape[0]
    w = types.SimpleNamespace(n_nodes=n, v_init=-65.0, area=area, cm=cm, clamp_off=None, clamp_amp=None,
                              clamp_freq=None, clamp_phase=None, globals=dict(W.DEFAULT_GLOBALS), dt=dt,
                              vmode="cable", slots=[], parent=parent, g_axial=g)
    m = oracle.Model(w)
    m.v[:], m.rhs[:], m.d[:] = v, rhs, d
    m.vcable()
    return m.v.copy()


def run_case(oracle, parent, area, g, cap, seed=0):
    rng = np.random.default_rng(seed)
    n = parent.shape[0]
    v = rng.uniform(-80.0, 20.0, n)
    rhs = rng.normal(0.0, 5.0, n)
    d = rng.uniform(0.0, 0.5, n)
    cm = rng.uniform(0.8, 1.2, n)
    dt = 0.025
    plan = mech.cable_plan(parent, cap)
    check_structure(plan, n, cap)
    got = replay(plan, v, rhs, d, cm, area, g, dt)
    want = oracle_step(oracle, parent, area, g, v, rhs, d, cm, dt)
    dv_got, dv_want = got - v, want - v
    scale = max(np.abs(dv_want).max(), 1e-300)
    err = np.abs(dv_got - dv_want).max() / scale
    assert err <= 1e-11, f"cap {cap}: max |ddv|/max|dv| = {err:.3g}"
    return plan


@pytest.mark.parametrize("cap", [1, 2, 5, 37, 200, 1000, 100000])
def test_random_cells_any_unit_bound(oracle, cap):
    parent, area, g = cells(11, [1, 3, 40, 700, 2500, 90])
    plan = run_case(oracle, parent.astype(np.int32), area, g, cap, seed=cap)
    if cap < 2500:
        assert np.any(plan["unit_mode"] == PIECE)


def test_long_chain_trunk_in_global_memory(oracle):
    parent = chain(600)
    rng = np.random.default_rng(3)
    area, g = geometry(rng, parent)
    plan = run_case(oracle, parent, area, g, 50)
    assert plan["list_top_g"].shape[0] == 1


def test_star_pieces_packed_into_forests(oracle):
    parent = np.concatenate([star(301), chain(40, 301)])
    rng = np.random.default_rng(4)
    area, g = geometry(rng, parent)
    plan = run_case(oracle, parent, area, g, 10)
    um, size = plan["unit_mode"], np.diff(plan["unit_pos"])
    # 300 one-node pieces share units of up to 10 nodes
    assert np.sum(um == PIECE) >= 30 and np.all(size[um == PIECE] <= 10)


def test_many_single_node_cells_share_units(oracle):
    parent = np.full(5000, -1, dtype=np.int32)
    rng = np.random.default_rng(5)
    area, g = geometry(rng, parent)
    plan = run_case(oracle, parent, area, g, 100000)
    assert plan["unit_mode"].shape[0] < 50


def test_config4_cells(oracle):
    w = W.make_config(4)
    sub, _ = W.cells_subset(w, list(range(0, 64, 4)))
    run_case(oracle, np.asarray(sub.parent, dtype=np.int32), sub.area, sub.g_axial, 4096)


def test_empty_and_invalid_trees():
    plan = mech.cable_plan(np.zeros(0, dtype=np.int32), 10)
    assert plan["unit_mode"].shape[0] == 0
    with pytest.raises(mech.MechError):
        mech.cable_plan(np.array([-1, 1], dtype=np.int32), 10)   # not Hines order
    with pytest.raises(mech.MechError):
        mech.cable_plan(np.array([-1, -1, 0], dtype=np.int32), 10)   # cell not contiguous
    with pytest.raises(mech.MechError):
        mech.cable_plan(np.array([-1, 0], dtype=np.int32), -1)
