"""Pins of the FP64 CPU oracle against facts fixed outside it.

Each test checks the oracle against a published value (tests/golden/), a
closed form of the mathematics, an invariant of the method, or brute force in
numpy, chosen so that a dropped term, a wrong sign, offset or index, or a
swapped operand in the oracle fails at least one of them.

Paper references: section 3 (BREAKPOINT current / conductance, DERIVATIVE +
SOLVE state update, density vs point-process mechanisms); section 5.2 (cnexp:
analytic solution with coefficients constant over a step; the numerically
approximated conductance).

Parity unpinned: the Ih and Ca-HVA rate constants are this project's own
synthetic definitions; beyond the closed forms and invariants below (their
limits, symmetric points, steady states and bounds) nothing external pins
them.
"""
import math
import os

import numpy as np
import pytest

from paper_1905_02241_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------------- hh --
def test_hh_resting_state_matches_textbook(oracle):
    m, h, n = oracle.hh_inf_tau(-65.0, 6.3)[:3]
    got = {"m_inf_rest": m, "h_inf_rest": h, "n_inf_rest": n}
    for name, val, tol in _golden("hh_resting_state.txt"):
        assert abs(got[name] - float(val)) <= float(tol), name


def test_hh_rates_at_their_reference_points(oracle):
    # exp(0) = 1 at the reference potential of every exponential rate
    r = oracle.hh_rates(-65.0)
    assert r[1] == 4.0 and r[2] == 0.07 and r[5] == 0.125
    assert oracle.hh_rates(-35.0)[3] == 0.5          # beta_h = 1/(1+1)
    # far from the singular points the vtrap rates approach their linear asymptote
    r = oracle.hh_rates(60.0)
    assert abs(r[0] - 0.1 * 100 / (1 - math.exp(-10))) < 1e-13
    assert abs(r[4] - 0.01 * 115 / (1 - math.exp(-11.5))) < 1e-15


def test_hh_removable_singularities(oracle):
    # alpha = a x/(1 - e^{-x/k}) -> a k at x = 0 (l'Hopital), and near it the
    # Bernoulli series a k (1 + u/2 + u^2/12), u = x/k
    assert oracle.hh_rates(-40.0)[0] == 1.0
    assert oracle.hh_rates(-55.0)[4] == 0.1
    for dx in (1e-9, -1e-9, 1e-6, -1e-6, 1e-3):
        u = dx / 10.0
        ser = 1 + u / 2 + u * u / 12
        assert abs(oracle.hh_rates(-40.0 + dx)[0] - ser) < 2e-15
        assert abs(oracle.hh_rates(-55.0 + dx)[4] - 0.1 * ser) < 2e-16


def _closed(name):
    return {r[0]: (float(r[1]), float(r[2])) for r in _golden("hh_syn_ca_closed_forms.txt")}[name]


def test_hh_time_constants_at_rest(oracle):
    got = oracle.hh_inf_tau(-65.0, 6.3)[3:]
    for name, g in zip(("tau_m_rest", "tau_h_rest", "tau_n_rest"), got):
        val, tol = _closed(name)
        assert abs(g - val) <= tol, name


def test_hh_gates_after_clamp_step_to_minus20(oracle):
    # away from -65 mV: beta_m, alpha_h and beta_n leave exp(0), so their
    # exponent scales (18, 20, 80 mV) and signs decide these values
    w = _single("hh", -20.0, 1000)
    M = oracle.Model(w)
    M.init()
    M.run(0, 1000)
    for k in "mhn":
        val, tol = _closed(f"{k}_clamp_minus20_1000")
        assert abs(M.states[0][k][0] - val) <= tol, k


def test_hh_net_current_at_rest(oracle):
    w = _single("hh", -65.0, 1)
    M = oracle.Model(w)
    M.init(-65.0)
    val, tol = _closed("i_hh_net_rest")
    assert abs(M.instance_current(0, 0, -65.0)[0] - val) <= tol


def test_mg_block_values(oracle):
    for v, name in ((-65.0, "mg_block_minus65"), (-20.0, "mg_block_minus20"), (0.0, "mg_block_0")):
        val, tol = _closed(name)
        assert abs(oracle.mg_block(v, 1.0) - val) <= tol, name


def test_synapse_peak_factor_values(oracle):
    for (tr, td), rec in (((0.2, 1.7), "ampa"), ((0.29, 43.0), "nmda")):
        f, tp = oracle.syn_peak_factor(tr, td)
        for got, name in ((f, f"f_{rec}"), (tp, f"tp_{rec}")):
            val, tol = _closed(name)
            assert abs(got - val) <= tol, name


def test_calcium_reversal_at_rest_concentration(oracle):
    val, tol = _closed("eca_cai0")
    assert abs(oracle.nernst_ca(5e-5, 2.0, 6.3) - val) <= tol


def test_q10_scales_time_constants_only(oracle):
    a = oracle.hh_inf_tau(-50.0, 6.3)
    b = oracle.hh_inf_tau(-50.0, 16.3)  # q10 = 3 exactly one decade up
    assert np.allclose(a[:3], b[:3], rtol=0, atol=0)
    assert np.allclose(a[3:] / 3.0, b[3:], rtol=1e-15)


def _single(kind, v_clamp, nsteps, params=None, dt=0.025, v_init=-65.0, **g):
    w = W.Workload("one", 1, [W._slot(kind, np.array([0]), params)], "clamp", dt, nsteps, v_init=v_init,
                   area=np.array([100.0]), cm=np.array([1.0]), clamp_off=np.array([v_clamp]),
                   clamp_amp=np.zeros(1), clamp_freq=np.zeros(1), clamp_phase=np.zeros(1))
    w.globals.update(g)
    return w


def test_cnexp_equals_closed_form_under_clamp(oracle):
    # With v held, x' = (x_inf - x)/tau has x(t) = x_inf + (x0 - x_inf) e^{-t/tau};
    # the cnexp iterate must reproduce it at every step to rounding.
    w = _single("hh", -20.0, 1000)
    M = oracle.Model(w)
    M.init()
    x0 = np.array([M.states[0][k][0] for k in "mhn"])
    inf_tau = oracle.hh_inf_tau(-20.0, 6.3)
    for block in range(4):
        M.run(block * 250, 250)
        t = (block + 1) * 250 * w.dt
        ref = inf_tau[:3] + (x0 - inf_tau[:3]) * np.exp(-t / inf_tau[3:])
        got = np.array([M.states[0][k][0] for k in "mhn"])
        assert np.all(np.abs(got - ref) <= 2e-15 + 1e-13 * np.abs(ref))


def test_steady_state_is_a_fixed_point(oracle):
    rng = np.random.default_rng(1)
    for kind in ("hh", "ih", "cahva"):
        for v in rng.uniform(-90, 30, 5):
            w = _single(kind, v, 50, v_init=v)
            if kind == "cahva":
                w.slots[0].params["gbar"][:] = 0.0   # keep cai at cai0
            M = oracle.Model(w)
            M.init(v)
            before = {k: a.copy() for k, a in M.states[0].items()}
            M.run(0, 50)
            for k, a in M.states[0].items():
                if kind == "cahva" and k == "cai":
                    continue
                assert np.array_equal(a, before[k]), (kind, k, v)


def test_gates_stay_in_unit_interval(oracle):
    w = W.make_tiny(3, kinds=("hh", "ih", "cahva"), n_nodes=40, shuffle=False, nsteps=400)
    w.clamp_amp[:] = 80.0   # swing the clamp over -145..15 mV
    M = oracle.Model(w)
    M.init()
    for _ in range(8):
        M.run(_ * 50, 50)
        for s, st in zip(w.slots, M.states):
            for name, a in st.items():
                if name != "cai":
                    assert np.all((a >= 0.0) & (a <= 1.0)), (s.kind, name)


# ----------------------------------------------------- currents and FD --
def test_current_vanishes_at_reversal(oracle):
    # pas at v = e; hh terms one at a time at their reversal; Ih at eh; synapse at e_syn
    w = _single("pas", 0.0, 1, params={"g": np.array([3e-3]), "e": np.array([-61.5])})
    M = oracle.Model(w)
    assert M.instance_current(0, 0, -61.5)[0] == 0.0
    w = _single("hh", 0.0, 1, params={"gkbar": np.array([0.0]), "gl": np.array([0.0])})
    M = oracle.Model(w)
    M.init()
    assert M.instance_current(0, 0, 50.0)[0] == 0.0          # ina at ena
    w = _single("hh", 0.0, 1, params={"gnabar": np.array([0.0]), "gl": np.array([0.0])})
    M = oracle.Model(w)
    M.init()
    assert M.instance_current(0, 0, -77.0)[0] == 0.0         # ik at ek
    w = _single("hh", 0.0, 1, params={"gnabar": np.array([0.0]), "gkbar": np.array([0.0])})
    M = oracle.Model(w)
    M.init()
    assert M.instance_current(0, 0, -54.3)[0] == 0.0         # il at el
    w = _single("ih", 0.0, 1)
    M = oracle.Model(w)
    M.init()
    assert M.instance_current(0, 0, -45.0)[0] == 0.0
    w = _single("syn", 0.0, 1)
    M = oracle.Model(w)
    M.init()
    for j, name in enumerate(("A_ampa", "B_ampa", "A_nmda", "B_nmda")):
        M.states[0][name][0] = [0.1, 0.7, 0.2, 0.9][j]
    assert M.instance_current(0, 0, 0.0)[0] == 0.0
    assert M.instance_current(0, 0, -65.0)[0] < 0.0          # inward at rest


def test_fd_conductance_matches_analytic(oracle):
    # ohmic currents: di/dv is the sum of the conductance products; the FD
    # error is rounding only, eps |i| / dv ~ 1e-11 relative
    w = _single("hh", 0.0, 1)
    M = oracle.Model(w)
    M.init(-30.0)
    m, h, n = (M.states[0][k][0] for k in "mhn")
    ga = 0.12 * m ** 3 * h + 0.036 * n ** 4 + 0.0003
    for v in (-80.0, -30.0, 10.0, 40.0):
        i, g = M.instance_current(0, 0, v)
        assert abs(g - ga) <= 1e-9 * ga
        # and i is linear in v with that slope
        assert abs(i - (0.12 * m ** 3 * h * (v - 50) + 0.036 * n ** 4 * (v + 77) + 0.0003 * (v + 54.3))) < 1e-13
    # NMDA: analytic g = 1e-3 (ga + gn (B + (v - e) B')), B' = 0.062 B (1 - B)
    w = _single("syn", 0.0, 1)
    M = oracle.Model(w)
    M.init()
    for name, val in zip(("A_ampa", "B_ampa", "A_nmda", "B_nmda"), (0.2, 1.0, 0.1, 0.6)):
        M.states[0][name][0] = val
    for v in (-70.0, -20.0, 5.0):
        B = 1.0 / (1.0 + math.exp(-0.062 * v) / 3.57)
        ga_an = 1e-3 * (0.8 + 0.5 * (B + v * 0.062 * B * (1 - B)))
        i, g = M.instance_current(0, 0, v)
        # O(dv) truncation of the forward difference: |i''| dv/2
        assert abs(g - ga_an) < 2e-7
        assert abs(i - 1e-3 * (0.8 + 0.5 * B) * v) < 1e-15


def test_mg_block_closed_forms(oracle):
    assert abs(oracle.mg_block(0.0, 1.0) - 3.57 / 4.57) < 4e-16   # two roundings apart
    assert oracle.mg_block(0.0, 0.0) == 1.0                 # no magnesium, no block
    vs = np.linspace(-120, 60, 50)
    b = np.array([oracle.mg_block(v, 1.0) for v in vs])
    assert np.all(np.diff(b) > 0) and b[0] < 3e-3 and b[-1] > 0.97


def test_synapse_peak_normalisation(oracle):
    for tr, td in ((0.2, 1.7), (0.29, 43.0)):
        f, tp = oracle.syn_peak_factor(tr, td)
        t = np.linspace(0, 10 * td, 2_000_001)
        g = f * (np.exp(-t / td) - np.exp(-t / tr))
        assert abs(g.max() - 1.0) < 1e-9
        assert abs(t[g.argmax()] - tp) < 2 * (t[1] - t[0])


def test_synapse_impulse_response(oracle):
    # a single event of weight w at step 0 gives g(t_n) = w f (e^{-t/td} - e^{-t/tr}) at t_n = n dt
    w = _single("syn", -65.0, 1, v_init=-65.0, params={"weight": np.array([1.7])})
    w.globals["event_rate_hz"] = 1e9    # p >= 1: fires at every step
    M = oracle.Model(w)
    M.init(-65.0)
    M.events(0)
    M.set_global("event_rate_hz", 0.0)
    fa, _ = oracle.syn_peak_factor(0.2, 1.7)
    fn, _ = oracle.syn_peak_factor(0.29, 43.0)
    st = M.states[0]
    assert st["A_ampa"][0] == st["B_ampa"][0] == 1.7 * fa
    for k in range(1, 401):
        M.run(k, 1)
        t = k * 0.025
        ga = st["B_ampa"][0] - st["A_ampa"][0]
        gn = st["B_nmda"][0] - st["A_nmda"][0]
        assert abs(ga - 1.7 * fa * (math.exp(-t / 1.7) - math.exp(-t / 0.2))) < 1e-13
        assert abs(gn - 1.7 * fn * (math.exp(-t / 43.0) - math.exp(-t / 0.29))) < 1e-13


def test_calcium_pool_relaxes_to_rest(oracle):
    w = _single("cahva", -65.0, 1, params={"gbar": np.array([0.0])})
    M = oracle.Model(w)
    M.init(-65.0)
    c0 = 3e-4
    M.states[0]["cai"][0] = c0
    M.run(0, 2000)
    t = 2000 * 0.025
    ref = 5e-5 + (c0 - 5e-5) * math.exp(-t / 80.0)
    assert abs(M.states[0]["cai"][0] - ref) < 1e-15


def test_calcium_influx_rate_from_si_units(oracle):
    # d cai/dt at cai = cai0 equals -kappa ica.  Independent SI derivation:
    # ica (mA/cm2) over 1 cm2 is ica*1e-3 A -> ica*1e-3/(2F) mol/s into a
    # shell of depth*1e-4 cm * 1 cm2 = depth*1e-7 L, free fraction gamma.
    F = 96485.33212
    gamma, depth = 0.05, 0.1
    ica = -2e-3
    mol_per_s = -ica * 1e-3 / (2 * F)
    mM_per_ms = gamma * mol_per_s / (depth * 1e-7) * 1e3 / 1e3
    assert abs(oracle.ca_kappa(gamma, depth) * -ica - mM_per_ms) < 1e-15 * mM_per_ms + 1e-20


def test_nernst_slope_matches_textbook(oracle):
    (celsius, slope, tol), = _golden("nernst_slope.txt")
    got = oracle.nernst_ca(1.0, 10.0, float(celsius))
    assert abs(got - float(slope)) <= float(tol)
    assert abs(oracle.nernst_ca(5e-5, 2.0, 6.3) - 1e3 * 8.314462618 * 279.45 / (2 * F_()) * math.log(4e4)) < 1e-10


def F_():
    return 96485.33212


# ------------------------------------------------------ Ih and Ca-HVA --
def test_ih_closed_forms(oracle):
    # alpha = beta at -90 mV: m_inf = 1/2 and tau = 1/(0.01) = 100 ms;
    # m_inf(v) = 1/(1 + e^{(v+90)/10}) by dividing alpha and beta
    mi, tau = oracle.ih_inf_tau(-90.0)
    assert mi == 0.5 and abs(tau - 100.0) < 1e-12
    for v in (-120.0, -70.0, -40.0):
        assert abs(oracle.ih_inf_tau(v)[0] - 1.0 / (1.0 + math.exp((v + 90) / 10))) < 1e-15


def test_cahva_closed_forms(oracle):
    # at v = -20 alpha_m hits its removable singularity (limit 0.5) and beta_h = 0.006/2
    o = oracle.cahva_inf_tau(-20.0)
    bm = 0.8 * math.exp(-25.0 / 15.0)
    assert abs(o[0] - 0.5 / (0.5 + bm)) < 1e-15
    ah = 0.0005 * math.exp(-40.0 / 25.0)
    assert abs(o[1] - ah / (ah + 0.003)) < 1e-15


# ------------------------------------------------------------- events --
def test_event_hash_matches_splitmix64_reference(oracle):
    for n, hx in _golden("splitmix64_seed0.txt"):
        # output number n of the stream seeded 0 is event draw (gid 0, k = n - 1)
        assert oracle.event_hash(0, 0, int(n) - 1) == int(hx, 16)


def test_event_rate_is_poisson(oracle):
    p_rate, dt = 5.0, 0.025
    T = oracle.event_threshold(p_rate, dt)
    assert T == math.floor(5.0 * 0.025 * 1e-3 * 2.0 ** 64)
    w = W.make_tiny(7, kinds=("syn",), n_nodes=2000, syn_per_node=5.0, event_rate_hz=200.0, vmode="clamp")
    M = oracle.Model(w)
    M.init()
    n_syn = w.slots[0].n
    fires = 0
    for k in range(200):
        M.states[0]["A_ampa"][:] = 0.0
        M.events(k)
        fires += int(np.count_nonzero(M.states[0]["A_ampa"]))
    p = 200.0 * 0.025e-3
    mean = p * n_syn * 200
    assert abs(fires - mean) < 5 * math.sqrt(mean)


# ------------------------------------------------------------ scatter --
def test_scatter_equals_numpy_add_at_bit_exact(oracle):
    # dyadic g, e, v, dv: every product and sum is exact, so the oracle's
    # rhs/d must equal numpy's unordered np.add.at bit for bit
    rng = np.random.default_rng(11)
    n_nodes = 37
    node = rng.integers(0, n_nodes, 300).astype(np.int32)
    g = rng.integers(1, 64, 300) * 2.0 ** -12
    e = rng.integers(-90, 10, 300).astype(float)
    w = W.Workload("scatter", n_nodes, [W._slot("pas", node, {"g": g, "e": e})], "external", 0.025, 1)
    w.globals["fd_dv"] = 2.0 ** -10
    M = oracle.Model(w)
    M.v[:] = rng.integers(-100, 40, n_nodes).astype(float)
    M.cur()
    rhs = np.zeros(n_nodes)
    d = np.zeros(n_nodes)
    np.add.at(rhs, node, -g * (M.v[node] - e))
    np.add.at(d, node, g)
    assert np.array_equal(M.rhs, rhs)
    assert np.array_equal(M.d, d)


def test_point_process_scatter_scales_by_area(oracle):
    w = W.make_tiny(5, kinds=("syn",), n_nodes=30, syn_per_node=4.0, shuffle=True)
    M = oracle.Model(w)
    M.init()
    rng = np.random.default_rng(2)
    for name in ("A_ampa", "B_ampa", "A_nmda", "B_nmda"):
        M.states[0][name][:] = rng.uniform(0, 2, w.slots[0].n)
    M.v[:] = rng.uniform(-80, 20, w.n_nodes)
    M.cur()
    node = w.slots[0].node
    I = np.array([M.instance_current(0, i, M.v[node[i]]) for i in range(w.slots[0].n)])
    rhs = np.zeros(w.n_nodes)
    d = np.zeros(w.n_nodes)
    np.add.at(rhs, node, -(1e2 / w.area[node]) * I[:, 0])
    np.add.at(d, node, (1e2 / w.area[node]) * I[:, 1])
    assert np.allclose(M.rhs, rhs, rtol=1e-13, atol=1e-18)
    assert np.allclose(M.d, d, rtol=1e-13, atol=1e-18)


# ------------------------------------------------------ voltage glue --
def test_isolated_backward_euler_closed_form(oracle):
    # pas only: v_{k+1} - e = (v_k - e) c/(c + g), c = 1e-3 cm/dt
    w = _single("pas", 0.0, 1, params={"g": np.array([2e-3]), "e": np.array([-70.0])})
    w.vmode = "isolated"
    w.cm = np.array([1.3])
    M = oracle.Model(w)
    M.init(-20.0)
    M.run(0, 200)
    c = 1e-3 * 1.3 / 0.025
    assert abs(M.v[0] - (-70.0 + 50.0 * (c / (c + 2e-3)) ** 200)) < 1e-12


def test_spike_count_equals_brute_force_crossings(oracle):
    w = W.make_tiny(9, kinds=("pas", "hh", "syn"), n_nodes=24, syn_per_node=6.0, vmode="isolated",
                    event_rate_hz=300.0, shuffle=False)
    w.area[:] = 100.0
    w.slots[-1].params["weight"][:] *= 8.0
    M = oracle.Model(w)
    M.init()
    R = oracle.Model(w)
    R.init()
    crossings = np.zeros(w.n_nodes, dtype=np.int64)
    for k in range(800):
        R.events(k)
        R.cur()
        v_old = R.v.copy()
        R.visolated()
        R.state()
        crossings += (v_old < -20.0) & (R.v >= -20.0)
    M.run(0, 800)
    assert crossings.sum() > 0
    assert np.array_equal(M.spikes, crossings)
    assert np.array_equal(M.v, R.v)


def test_clamp_waveform(oracle):
    w = W.make_tiny(4, kinds=("pas",), n_nodes=10)
    M = oracle.Model(w)
    t = 3.725
    M.vclamp(t)
    ref = w.clamp_off + w.clamp_amp * np.sin(2 * np.pi * w.clamp_freq * t / 1000 + w.clamp_phase)
    assert np.allclose(M.v, ref, rtol=0, atol=1e-12)


# -------------------------------------- section 5.2 variants (F1, F2) --
def test_analytic_conductance_matches_central_difference(oracle):
    """CONDUCTANCE variant: the closed-form di/dv equals a central difference
    of the oracle's own current (h = 1e-4 mV, error O(h^2)) for every type."""
    w = W.make_tiny(21, n_nodes=12, per_node=1, syn_per_node=3.0, vmode="external")
    w.globals["analytic_conductance"] = 1
    M = oracle.Model(w)
    M.init()
    rng = np.random.default_rng(4)
    for s, sl in enumerate(w.slots):
        if sl.kind == "syn":
            for name in M.states[s]:
                M.states[s][name][:] = rng.uniform(0, 3, sl.n)
        for i in range(sl.n):
            for v in (-75.0, -30.0, 15.0):
                _, g = M.instance_current(s, i, v)
                ip, _ = M.instance_current(s, i, v + 1e-4)
                im, _ = M.instance_current(s, i, v - 1e-4)
                cd = (ip - im) / 2e-4
                assert abs(g - cd) <= 1e-7 * (abs(cd) + abs(g)) + 1e-15, (sl.kind, v)


def test_analytic_conductance_leaves_rhs_and_states(oracle):
    """Only d changes with the CONDUCTANCE variant: rhs and every STATE are
    bit-identical, d agrees with the finite difference to O(dv)."""
    w = W.make_tiny(22, per_node=2, nsteps=40)
    A = oracle.Model(w)
    A.init()
    A.run(0, 40)
    w.globals["analytic_conductance"] = 1
    B = oracle.Model(w)
    B.init()
    B.run(0, 40)
    assert np.array_equal(A.rhs, B.rhs)
    for s in range(len(w.slots)):
        for name in A.states[s]:
            assert np.array_equal(A.states[s][name], B.states[s][name])
    assert np.allclose(A.d, B.d, rtol=2e-4, atol=1e-12)


def _pade(y):
    return (1 - y / 2) / (1 + y / 2)


def test_pade_cnexp_is_geometric_under_clamp(oracle):
    """Pade variant: with v held the iterate is x_inf + (x0 - x_inf) P(dt/tau)^n,
    P(y) = (1 - y/2)/(1 + y/2)."""
    w = _single("hh", -20.0, 400)
    w.globals["pade_cnexp"] = 1
    M = oracle.Model(w)
    M.init()
    x0 = np.array([M.states[0][k][0] for k in "mhn"])
    it = oracle.hh_inf_tau(-20.0, 6.3)
    M.run(0, 400)
    ref = it[:3] + (x0 - it[:3]) * _pade(0.025 / it[3:]) ** 400
    got = np.array([M.states[0][k][0] for k in "mhn"])
    assert np.all(np.abs(got - ref) <= 1e-14 + 1e-12 * np.abs(ref))


def test_pade_cnexp_error_within_its_bound(oracle):
    """One step: |P(y) - e^-y| <= y^3/12 (the leading error term of the (1,1)
    approximant, an upper bound for 0 < y < 1), scaled by |x - x_inf|."""
    for v in (-70.0, -40.0, 0.0, 30.0):
        w = _single("hh", v, 1)
        E = oracle.Model(w)
        E.init()
        w2 = _single("hh", v, 1)
        w2.globals["pade_cnexp"] = 1
        P = oracle.Model(w2)
        P.init()
        it = oracle.hh_inf_tau(v, 6.3)
        E.run(0, 1)
        P.run(0, 1)
        for j, k in enumerate("mhn"):
            y = 0.025 / it[3 + j]
            x0 = oracle.hh_inf_tau(-65.0, 6.3)[j]
            bound = y ** 3 / 12 * abs(x0 - it[j]) + 1e-15
            assert abs(E.states[0][k][0] - P.states[0][k][0]) <= bound, (v, k)


def test_pade_keeps_fixed_points_and_bounds(oracle):
    w = W.make_tiny(23, kinds=("hh", "ih", "cahva"), n_nodes=30, shuffle=False, nsteps=300)
    w.globals["pade_cnexp"] = 1
    w.clamp_amp[:] = 70.0
    M = oracle.Model(w)
    M.init()
    M.run(0, 300)
    for st in M.states:
        for name, a in st.items():
            if name != "cai":
                assert np.all((a >= 0) & (a <= 1))
    v = -48.0
    w = _single("hh", v, 30, v_init=v)
    w.globals["pade_cnexp"] = 1
    M = oracle.Model(w)
    M.init(v)
    before = {k: a.copy() for k, a in M.states[0].items()}
    M.run(0, 30)
    for k in before:
        assert np.array_equal(before[k], M.states[0][k])


def test_pade_synapse_decay(oracle):
    w = _single("syn", -65.0, 1, params={"weight": np.array([2.0])})
    w.globals["pade_cnexp"] = 1
    w.globals["event_rate_hz"] = 1e9
    M = oracle.Model(w)
    M.init(-65.0)
    M.events(0)
    M.set_global("event_rate_hz", 0.0)
    a0 = M.states[0]["B_nmda"][0]
    M.run(1, 200)
    assert abs(M.states[0]["B_nmda"][0] - a0 * _pade(0.025 / 43.0) ** 200) < 1e-14 * a0


# ------------------------------------- implicit solves (F3): kmarkov, capump --
def test_kmarkov_matrix_conserves_probability(oracle):
    """I - dt A with a generator A (columns summing to zero): every column of
    the implicit Euler matrix sums to one, so C1 + C2 + O is conserved."""
    for v in (-90.0, -55.0, -20.0, 30.0):
        M = oracle.kmarkov_matrix(v, 6.3, 0.025)
        assert np.allclose(M.sum(axis=0), 1.0, rtol=0, atol=1e-15)
        assert np.all(np.diag(M) >= 1.0) and np.all(M - np.diag(np.diag(M)) <= 0)


def test_kmarkov_step_equals_library_solve(oracle):
    rng = np.random.default_rng(8)
    for v in rng.uniform(-100, 50, 20):
        x = rng.dirichlet(np.ones(3))
        ref = np.linalg.solve(oracle.kmarkov_matrix(v, 6.3, 0.025), x)
        got = oracle.kmarkov_step(v, 6.3, 0.025, x)
        assert np.allclose(got, ref, rtol=1e-14, atol=1e-16)
        assert abs(got.sum() - 1.0) < 4e-16


def test_kmarkov_equilibrium_is_binomial_fixed_point(oracle):
    for v in (-80.0, -40.0, 10.0):
        n = oracle.hh_inf_tau(v, 6.3)[2]
        x = np.array([(1 - n) ** 2, 2 * n * (1 - n), n * n])
        y = oracle.kmarkov_step(v, 6.3, 0.025, x)
        assert np.allclose(y, x, rtol=0, atol=2e-16)


def test_kmarkov_converges_to_two_gate_solution(oracle):
    """The scheme C1 <-(2a,b)-> C2 <-(a,2b)-> O is two independent n-gates:
    from a binomial start the exact O(t) is n(t)^2 with n(t) the HH gate.
    Implicit Euler approaches it at first order in dt."""
    v0, v1, T = -65.0, -10.0, 2.0
    n0 = oracle.hh_inf_tau(v0, 6.3)[2]
    ninf, tau = oracle.hh_inf_tau(v1, 6.3)[2], oracle.hh_inf_tau(v1, 6.3)[5]
    exact = (ninf + (n0 - ninf) * math.exp(-T / tau)) ** 2
    errs = []
    for dt in (0.02, 0.01, 0.005):
        x = np.array([(1 - n0) ** 2, 2 * n0 * (1 - n0), n0 * n0])
        for _ in range(int(round(T / dt))):
            x = oracle.kmarkov_step(v1, 6.3, dt, x)
        errs.append(abs(x[2] - exact))
    assert errs[0] < 2e-3
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


def test_capump_newton_solves_implicit_equation(oracle):
    """derivimplicit: four Newton steps reach the root of the implicit Euler
    equation; scipy's bracketing root finder on the same equation agrees."""
    from scipy.optimize import brentq
    w = _single("capump", -65.0, 1)
    M = oracle.Model(w)
    kappa = oracle.ca_kappa(0.05, 0.1)
    vmax, kp, c0r = 1e-4, 1e-3, 5e-5
    F = lambda c, ica: -kappa * ica - vmax * (c / (c + kp) - c0r / (c0r + kp))
    for ica, c in ((-2e-3, 5e-5), (-1e-2, 3e-3), (0.0, 2e-3), (-5e-4, 1e-6)):
        got, res = M.capump_step(ica, c, 4)
        assert abs(res) <= 1e-18 + 1e-15 * got
        ref = brentq(lambda x: x - c - 0.025 * F(x, ica), 1e-12, 1.0, xtol=1e-22, rtol=9e-16)
        assert abs(got - ref) <= 4e-15 * ref


def test_capump_reduces_to_linear_implicit_euler(oracle):
    """vmax = 0: F is constant, so implicit Euler is c + dt(-kappa ica)."""
    w = _single("capump", -65.0, 1)
    w.globals["pump_vmax"] = 0.0
    M = oracle.Model(w)
    kappa = oracle.ca_kappa(0.05, 0.1)
    got, _ = M.capump_step(-3e-3, 1e-4, 4)
    assert abs(got - (1e-4 + 0.025 * kappa * 3e-3)) < 1e-18


def test_capump_rest_is_fixed_point_and_relaxation_monotone(oracle):
    w = _single("capump", -65.0, 1)
    M = oracle.Model(w)
    got, _ = M.capump_step(0.0, 5e-5, 4)
    assert got == 5e-5
    c = 2e-3
    prev = c
    for _ in range(200):
        c, _ = M.capump_step(0.0, c, 4)
        assert 5e-5 < c < prev
        prev = c


def test_new_kinds_vanish_at_reversal(oracle):
    w = _single("kmarkov", 0.0, 1)
    M = oracle.Model(w)
    M.init()
    assert M.instance_current(0, 0, -77.0)[0] == 0.0
    w = _single("capump", 0.0, 1)
    M = oracle.Model(w)
    M.init()
    eca = oracle.nernst_ca(5e-5, 2.0, 6.3)
    assert M.instance_current(0, 0, eca)[0] == 0.0


# -------------------------------------------- cable mode: Hines solve (F4) --
def _cable_matrix(M, dt):
    """Dense matrix and right-hand side of the linearised backward Euler step,
    assembled independently of the tree elimination."""
    n = M.n_nodes
    A = np.diag(1e-3 * M.cm / dt + M.d)
    r = M.rhs.copy()
    for i in range(n):
        p = M.parent[i]
        if p < 0:
            continue
        ki, kp = 1e2 * M.g_axial[i] / M.area[i], 1e2 * M.g_axial[i] / M.area[p]
        A[i, i] += ki
        A[p, p] += kp
        A[i, p] -= ki
        A[p, i] -= kp
        r[i] += ki * (M.v[p] - M.v[i])
        r[p] += kp * (M.v[i] - M.v[p])
    return A, r


def test_hines_solve_equals_dense_library_solve(oracle):
    w = W.make_cells(3, n_cells=3, lo=20, hi=60, nsteps=1)
    M = oracle.Model(w)
    M.init()
    rng = np.random.default_rng(5)
    M.v[:] = rng.uniform(-80, 20, w.n_nodes)
    M.events(0)
    M.cur()
    A, r = _cable_matrix(M, w.dt)
    ref = M.v + np.linalg.solve(A, r)
    M.vcable()
    assert np.allclose(M.v, ref, rtol=1e-13, atol=1e-11)


def test_cable_without_coupling_is_isolated(oracle):
    w = W.make_cells(4, n_cells=2, lo=30, hi=40, nsteps=200)
    w.g_axial[:] = 0.0
    A = oracle.Model(w)
    A.init()
    A.run(0, 200, "cable")
    B = oracle.Model(w)
    B.init()
    B.run(0, 200, "isolated")
    assert np.array_equal(A.v, B.v)
    assert np.array_equal(A.spikes, B.spikes)


def test_cable_conserves_charge_without_membrane_current(oracle):
    """With no mechanism (rhs = d = 0) the axial currents only move charge:
    sum_n area_n cm_n dv_n = 0, and a uniform potential stays uniform."""
    w = W.make_cells(5, n_cells=2, lo=40, hi=80, kinds=(), nsteps=1)
    M = oracle.Model(w)
    rng = np.random.default_rng(6)
    M.v[:] = rng.uniform(-90, 30, w.n_nodes)
    q0 = np.sum(w.area * M.v)
    for _ in range(50):
        M.rhs[:] = 0.0
        M.d[:] = 0.0
        M.vcable()
    assert abs(np.sum(w.area * M.v) - q0) <= 1e-9 * np.sum(w.area)
    M.v[:] = -42.0
    M.rhs[:] = 0.0
    M.d[:] = 0.0
    M.vcable()
    assert np.all(M.v == -42.0)


def test_cable_spreads_current_along_the_tree(oracle):
    """Two compartments: the closed-form 2x2 solve."""
    w = W.Workload("two", 2, [], "cable", 0.025, 1, area=np.array([100.0, 50.0]), cm=np.array([1.0, 1.0]),
                   parent=np.array([-1, 0], dtype=np.int32), g_axial=np.array([0.0, 0.02]))
    M = oracle.Model(w)
    M.v[:] = [-65.0, -20.0]
    M.rhs[:] = [0.3, -0.1]
    M.d[:] = [0.01, 0.002]
    c = 1e-3 / 0.025
    k0, k1 = 1e2 * 0.02 / 100.0, 1e2 * 0.02 / 50.0
    a = np.array([[c + 0.01 + k0, -k0], [-k1, c + 0.002 + k1]])
    r = np.array([0.3 + k0 * 45.0, -0.1 - k1 * 45.0])
    det = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
    dv = np.array([(r[0] * a[1, 1] - a[0, 1] * r[1]) / det, (a[0, 0] * r[1] - a[1, 0] * r[0]) / det])
    M.vcable()
    assert np.allclose(M.v, np.array([-65.0, -20.0]) + dv, rtol=0, atol=1e-12)


# ------------------------------------ per-node calcium ion, USEION (F4) --
def _ca_mesh(seed, kinds, per_node, vmode, gbar=None, frac=0.7):
    w = W.make_tiny(seed, kinds=kinds, n_nodes=60, per_node=per_node, vmode=vmode, nsteps=300,
                    shuffle=False, density_fraction=frac)
    if gbar is not None:
        for s in w.slots:
            if s.kind in ("cahva", "capump"):
                s.params["gbar"][:] = gbar(s.n)
    return w


def _run(oracle, w, shared, nsteps=300):
    w.globals["shared_ca"] = shared
    M = oracle.Model(w)
    M.init()
    M.run(0, nsteps)
    return M


def test_shared_calcium_with_one_channel_per_node_is_the_own_pool(oracle):
    """One Ca-HVA instance per node: the node's pool sees exactly that
    instance's current (0 + ica), so the shared ion reproduces the
    per-instance pool bit for bit; nodes without a calcium channel keep
    cai0 exactly."""
    w = _ca_mesh(81, ("pas", "hh", "cahva"), 1, "isolated")
    own = _run(oracle, w, 0)
    shared = _run(oracle, w, 1)
    s = [i for i, sl in enumerate(w.slots) if sl.kind == "cahva"][0]
    node = w.slots[s].node
    assert np.array_equal(own.v, shared.v)
    assert np.array_equal(own.states[s]["m"], shared.states[s]["m"])
    assert np.array_equal(own.states[s]["cai"], shared.cai_node[node])
    rest = np.setdiff1d(np.arange(w.n_nodes), node)
    assert rest.size > 0 and np.all(shared.cai_node[rest] == w.globals["cai0"])
    assert np.all(shared.cai_node[node] != w.globals["cai0"])


def test_shared_calcium_sums_channels_on_a_node(oracle):
    """Two Ca-HVA instances with equal gates on a node (same v, same initial
    state) and conductances g1, g2 feed one pool: the same as one instance of
    g1 + g2, up to the rounding of the split product.  Without the shared ion
    each instance's own pool sees half the influx, a different result."""
    import copy
    two = _ca_mesh(82, ("cahva",), 2, "clamp")
    node = two.slots[0].node
    assert np.array_equal(node[::2], node[1::2])
    g = two.slots[0].params["gbar"]
    one = copy.deepcopy(two)
    one.slots[0] = W._slot("cahva", node[::2].copy(), {"gbar": g[::2] + g[1::2]})
    a = _run(oracle, two, 1)
    b = _run(oracle, one, 1)
    assert np.allclose(a.cai_node, b.cai_node, rtol=1e-12, atol=0.0)
    assert np.allclose(a.rhs, b.rhs, rtol=1e-12, atol=1e-18)
    own = _run(oracle, two, 0)
    assert np.max(np.abs(own.states[0]["cai"] - a.cai_node[node]) / a.cai_node[node]) > 1e-3


def test_shared_calcium_capump_channel_feeds_the_linear_pool(oracle):
    """Under the shared ion a capump instance contributes its channel current
    (the Ca-HVA gates and current) and the node's pool follows the linear
    law: one capump per node then equals Ca-HVA with its own pool exactly."""
    wa = _ca_mesh(83, ("pas", "capump"), 1, "isolated")
    wb = _ca_mesh(83, ("pas", "cahva"), 1, "isolated")
    for s in wb.slots:
        if s.kind == "cahva":
            s.params["gbar"][:] = [x for x in wa.slots if x.kind == "capump"][0].params["gbar"]
    a = _run(oracle, wa, 1)
    b = _run(oracle, wb, 0)
    sb = [i for i, sl in enumerate(wb.slots) if sl.kind == "cahva"][0]
    assert np.array_equal(a.v, b.v)
    assert np.array_equal(a.cai_node[wb.slots[sb].node], b.states[sb]["cai"])


# ------------------- derivimplicit on a coupled 2x2 system: cabuf (F3) --
def _cabuf_F(c, b, ica, btot=0.05, kon=100.0, koff=0.1, kappa=None, tau=80.0, c0r=5e-5):
    bind = kon * c * (btot - b) - koff * b
    return np.array([-kappa * ica - bind - (c - c0r) / tau, bind])


def test_cabuf_newton_solves_the_coupled_implicit_equation(oracle):
    """Free and buffer-bound calcium, implicit Euler: the Newton steps reach
    the root of the 2x2 system; scipy's hybrid root finder on the same
    equations, written here from the rates, agrees."""
    from scipy.optimize import root
    w = _single("cabuf", -65.0, 1)
    M = oracle.Model(w)
    kappa = oracle.ca_kappa(0.05, 0.1)
    for ica, c, b in ((-2e-3, 5e-5, 2e-3), (-2e-2, 3e-3, 0.04), (0.0, 2e-3, 1e-3), (-5e-4, 1e-6, 0.0)):
        gc, gb, res = M.cabuf_step(ica, c, b, 6)
        assert res <= 1e-18
        G = lambda x: x - np.array([c, b]) - 0.025 * _cabuf_F(x[0], x[1], ica, kappa=kappa)
        ref = root(G, [c, b], method="hybr", tol=1e-16).x
        assert abs(gc - ref[0]) <= 1e-13 * ref[0] and abs(gb - ref[1]) <= 1e-13 * max(ref[1], 1e-6)


def test_cabuf_newton_converges_quadratically(oracle):
    """Newton with the exact Jacobian squares the error each step; a wrong
    Jacobian entry would leave linear convergence."""
    w = _single("cabuf", -65.0, 1)
    M = oracle.Model(w)
    res = [M.cabuf_step(-5e-2, 1e-3, 1e-3, k, dt=1.0)[2] for k in (1, 2, 3)]
    assert res[0] > 1e-8
    assert res[1] <= 50.0 * res[0] ** 2 / 5e-3 and res[2] <= 50.0 * res[1] ** 2 / 5e-3 + 1e-18
    assert res[2] < 1e-6 * res[0]


def test_cabuf_without_buffer_is_linear_implicit_euler(oracle):
    """btot = 0 and no bound calcium: the pool is linear, and implicit Euler
    has the closed form c = (c_old + dt(-kappa ica + cai0/tau))/(1 + dt/tau)."""
    w = _single("cabuf", -65.0, 1, buf_total=0.0)
    M = oracle.Model(w)
    kappa = oracle.ca_kappa(0.05, 0.1)
    gc, gb, _ = M.cabuf_step(-3e-3, 1e-4, 0.0, 4)
    ref = (1e-4 + 0.025 * (kappa * 3e-3 + 5e-5 / 80.0)) / (1.0 + 0.025 / 80.0)
    assert gb == 0.0 and abs(gc - ref) <= 2e-16 * ref


def test_cabuf_conserves_calcium_without_influx_or_extrusion(oracle):
    """ica = 0 and no extrusion (tau_ca very large): binding only moves
    calcium between free and bound, so c + b is kept, and the pool settles at
    the binding equilibrium b/(btot - b) = kon c/koff."""
    w = _single("cabuf", -65.0, 1, tau_ca=1e30)
    M = oracle.Model(w)
    c, b = 2e-3, 1e-3
    total = c + b
    for _ in range(400):
        c, b, _ = M.cabuf_step(0.0, c, b, 4)
        assert abs(c + b - total) <= 1e-15 * total
    assert abs(b * 0.1 - 100.0 * c * (0.05 - b)) <= 1e-12 * 100.0 * c * 0.05
    assert abs(M.cabuf_bound(c) - b) <= 1e-12 * b


def test_cabuf_rest_is_a_fixed_point(oracle):
    w = _single("cabuf", -65.0, 1)
    M = oracle.Model(w)
    b0 = M.cabuf_bound(5e-5)
    assert abs(b0 - 0.05 * 5e-5 / (5e-5 + 1e-3)) <= 1e-17
    gc, gb, res = M.cabuf_step(0.0, 5e-5, b0, 4)
    assert abs(gc - 5e-5) <= 1e-20 and abs(gb - b0) <= 1e-18
