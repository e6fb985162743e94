/*
 * mech_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Straight scalar loops in the order of the timestep described in
 * mech_oracle.h.  Built with -O2 -fno-fast-math -ffp-contract=off against the
 * host libm, single threaded, so the summation order of rhs/d is the instance
 * order and every rounding is an IEEE double rounding.
 *
 * Paper references:
 *   section 3 (NMODL DSL): SUFFIX density mechanisms vs POINT_PROCESS
 *     synapses, RANGE / PARAMETER / ASSIGNED / STATE variables, BREAKPOINT
 *     (current and conductance each step), DERIVATIVE + SOLVE (state update);
 *   section 5.2 (SymPy): linear independent ODEs are advanced by their analytic
 *     solution with the coefficients held constant over the step (cnexp);
 *   section 5.2, last paragraph: by default the conductance di/dv is
 *     approximated numerically at run time;
 *   section 8, Table 3: a timestep is State Update + Current Update + Other.
 *
 * Mechanism equations (the paper gives none; these are readings of its names):
 *   hh    Hodgkin & Huxley (1952) kinetics, modern sign convention, rest -65 mV
 *   pas   i = g (v - e)
 *   ih    one gate, alpha = 0.005 exp(-(v+90)/20), beta = 0.005 exp((v+90)/20)
 *   cahva m^2 h, Nernst eca, shell calcium with relaxation to cai0
 *   syn   double-exponential AMPA + NMDA conductance with Mg block
 *   kmarkov  three-state C1-C2-O potassium scheme, implicit Euler (sparse)
 *   capump   Ca-HVA gates with a pool emptied by a saturable pump, implicit
 *            Euler solved by Newton's method (derivimplicit)
 *   cabuf    Ca-HVA gates with free and buffer-bound calcium, implicit Euler
 *            solved by Newton's method on the 2x2 system (derivimplicit)
 *   shared_ca  calcium as a per-node ion (USEION, section 3): the calcium
 *            currents of all instances on a node feed one pool per node
 */
#include "mech_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define ORC_PI 3.14159265358979323846
#define ORC_R 8.314462618   /* J/(mol K) */
#define ORC_F 96485.33212   /* C/mol     */

/* ------------------------------------------------------------------ hh -- */
/* Hodgkin-Huxley rate functions, 1/ms at q10 = 1.  alpha_m and alpha_n have a
 * removable singularity (0/0) at v = -40 and v = -55; the value there is the
 * limit, and expm1 keeps the denominator accurate next to it.               */
static double hh_am(double v) {
    double x = v + 40.0;
    if (x == 0.0) return 1.0;
    return 0.1 * x / (-expm1(-x / 10.0));
}
static double hh_bm(double v) { return 4.0 * exp(-(v + 65.0) / 18.0); }
static double hh_ah(double v) { return 0.07 * exp(-(v + 65.0) / 20.0); }
static double hh_bh(double v) { return 1.0 / (1.0 + exp(-(v + 35.0) / 10.0)); }
static double hh_an(double v) {
    double x = v + 55.0;
    if (x == 0.0) return 0.1;
    return 0.01 * x / (-expm1(-x / 10.0));
}
static double hh_bn(double v) { return 0.125 * exp(-(v + 65.0) / 80.0); }

static double hh_q10(double celsius) { return pow(3.0, (celsius - 6.3) / 10.0); }

void orc_hh_rates(double v, double *o) {
    o[0] = hh_am(v); o[1] = hh_bm(v);
    o[2] = hh_ah(v); o[3] = hh_bh(v);
    o[4] = hh_an(v); o[5] = hh_bn(v);
}

void orc_hh_inf_tau(double v, double celsius, double *o) {
    double r[6], q = hh_q10(celsius);
    orc_hh_rates(v, r);
    for (int j = 0; j < 3; ++j) {
        double a = r[2 * j], b = r[2 * j + 1];
        o[j] = a / (a + b);
        o[3 + j] = 1.0 / (q * (a + b));
    }
}

/* ------------------------------------------------------------------ ih -- */
static double ih_a(double v) { return 0.005 * exp(-(v + 90.0) / 20.0); }
static double ih_b(double v) { return 0.005 * exp((v + 90.0) / 20.0); }

void orc_ih_inf_tau(double v, double *o) {
    double a = ih_a(v), b = ih_b(v);
    o[0] = a / (a + b);
    o[1] = 1.0 / (a + b);
}

/* --------------------------------------------------------------- cahva -- */
static double ca_am(double v) {
    double x = v + 20.0;
    if (x == 0.0) return 0.5;
    return 0.1 * x / (-expm1(-x / 5.0));
}
static double ca_bm(double v) { return 0.8 * exp(-(v + 45.0) / 15.0); }
static double ca_ah(double v) { return 0.0005 * exp(-(v + 60.0) / 25.0); }
static double ca_bh(double v) { return 0.006 / (1.0 + exp(-(v + 20.0) / 10.0)); }

void orc_cahva_inf_tau(double v, double *o) {
    double am = ca_am(v), bm = ca_bm(v), ah = ca_ah(v), bh = ca_bh(v);
    o[0] = am / (am + bm);
    o[1] = ah / (ah + bh);
    o[2] = 1.0 / (am + bm);
    o[3] = 1.0 / (ah + bh);
}

/* ------------------------------------------------------------- kmarkov -- */
/* Three-state potassium scheme C1 <-> C2 <-> O with the Hodgkin-Huxley n-gate
 * rates a = q10 alpha_n, b = q10 beta_n:  C1 -> C2 at 2a, C2 -> C1 at b,
 * C2 -> O at a, O -> C2 at 2b.  Its equilibrium is the binomial
 * (1-n)^2, 2n(1-n), n^2 with n = n_inf, so O plays the role of n^2.
 * dx/dt = A x; implicit Euler solves (I - dt A) x_new = x_old.            */
void orc_kmarkov_matrix(double v, double celsius, double dt, double *M) {
    double q = hh_q10(celsius);
    double a = q * hh_an(v), b = q * hh_bn(v);
    double A[9] = {-2.0 * a, b, 0.0,
                   2.0 * a, -(a + b), 2.0 * b,
                   0.0, a, -2.0 * b};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            M[3 * r + c] = (r == c ? 1.0 : 0.0) - dt * A[3 * r + c];
}

/* Gaussian elimination with partial pivoting on a 3x3 system (textbook). */
/* M x = b for n <= 4 by Gaussian elimination with partial pivoting (row
 * major M, x holds b on entry and the solution on return).                 */
static void solve_n(int n, double *M, double *x) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(M[n * r + k]) > fabs(M[n * p + k])) p = r;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = M[n * k + c]; M[n * k + c] = M[n * p + c]; M[n * p + c] = t;
            }
            double t = x[k]; x[k] = x[p]; x[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double f = M[n * r + k] / M[n * k + k];
            for (int c = k; c < n; ++c) M[n * r + c] -= f * M[n * k + c];
            x[r] -= f * x[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double sum = x[k];
        for (int c = k + 1; c < n; ++c) sum -= M[n * k + c] * x[c];
        x[k] = sum / M[n * k + k];
    }
}

void orc_kmarkov_step(double v, double celsius, double dt, double *x) {
    double M[9];
    orc_kmarkov_matrix(v, celsius, dt, M);
    solve_n(3, M, x);
}

/* -------------------------------------------------------------- capump -- */
static double pump_rate(const orc_globals *gl, double c) {
    return gl->pump_vmax * (c / (c + gl->pump_kp) - gl->cai0 / (gl->cai0 + gl->pump_kp));
}

double orc_capump_step(const orc_globals *gl, double ica, double dt, double *cai, int iters) {
    double kappa = orc_ca_kappa(gl->ca_gamma, gl->ca_depth);
    double c0 = *cai, c = c0, G = 0.0;
    for (int it = 0; it < iters; ++it) {
        double F = -kappa * ica - pump_rate(gl, c);
        double dF = -gl->pump_vmax * gl->pump_kp / ((c + gl->pump_kp) * (c + gl->pump_kp));
        G = c - c0 - dt * F;
        c = c - G / (1.0 - dt * dF);
    }
    *cai = c;
    return c - c0 - dt * (-kappa * ica - pump_rate(gl, c));
}

/* --------------------------------------------------------------- cabuf -- */
/* Free calcium c and buffer-bound calcium b (total buffer btot, binding
 * kon c (btot - b), unbinding koff b) in a pool that relaxes to cai0:
 *   dc/dt = -kappa ica - kon c (btot - b) + koff b - (c - cai0)/tau_ca
 *   db/dt =  kon c (btot - b) - koff b
 * Implicit Euler (the derivimplicit method, section 5.2) gives
 * G(c, b) = (c - c_old - dt F_c, b - b_old - dt F_b) = 0, solved by `iters`
 * Newton steps from the old state with the analytic Jacobian
 * I - dt dF/d(c, b); each step solves the 2x2 system.  Returns the max-norm
 * of G at the result.                                                       */
static void cabuf_rates(const orc_globals *gl, double kappa, double ica, double c, double b, double *F) {
    double bind = gl->buf_kon * c * (gl->buf_total - b) - gl->buf_koff * b;
    F[0] = -kappa * ica - bind - (c - gl->cai0) / gl->tau_ca;
    F[1] = bind;
}

double orc_cabuf_step(const orc_globals *gl, double ica, double dt, double *cai, double *cab, int iters) {
    double kappa = orc_ca_kappa(gl->ca_gamma, gl->ca_depth);
    double c0 = *cai, b0 = *cab, c = c0, b = b0, F[2];
    for (int it = 0; it < iters; ++it) {
        cabuf_rates(gl, kappa, ica, c, b, F);
        double G[2] = {-(c - c0 - dt * F[0]), -(b - b0 - dt * F[1])};
        double dbind_dc = gl->buf_kon * (gl->buf_total - b), dbind_db = -gl->buf_kon * c - gl->buf_koff;
        double J[4] = {1.0 - dt * (-dbind_dc - 1.0 / gl->tau_ca), -dt * (-dbind_db),
                       -dt * dbind_dc, 1.0 - dt * dbind_db};
        solve_n(2, J, G);
        c += G[0];
        b += G[1];
    }
    *cai = c;
    *cab = b;
    cabuf_rates(gl, kappa, ica, c, b, F);
    double r0 = fabs(c - c0 - dt * F[0]), r1 = fabs(b - b0 - dt * F[1]);
    return r0 > r1 ? r0 : r1;
}

/* the bound calcium in equilibrium with free calcium c                     */
double orc_cabuf_bound(const orc_globals *gl, double c) {
    return gl->buf_total * gl->buf_kon * c / (gl->buf_kon * c + gl->buf_koff);
}

double orc_nernst_ca(double cai, double cao, double celsius) {
    double T = celsius + 273.15;
    return 1e3 * ORC_R * T / (2.0 * ORC_F) * log(cao / cai);
}

/* d cai/dt = -kappa*ica - (cai - cai0)/tau_ca.  A current density ica
 * (mA/cm2) carries ica*1e-3/(2F) mol/(s cm2) into a shell of depth `depth` um
 * (depth*1e-7 L per cm2), of which the fraction gamma stays free:
 * kappa = 1e4*gamma/(2*F*depth) in mM/ms per mA/cm2.                        */
double orc_ca_kappa(double gamma, double depth) {
    return 1e4 * gamma / (2.0 * ORC_F * depth);
}

/* ----------------------------------------------------------------- syn -- */
double orc_mg_block(double v, double mg) {
    return 1.0 / (1.0 + exp(-0.062 * v) * mg / 3.57);
}

/* g(t) = exp(-t/tau_d) - exp(-t/tau_r) peaks at
 * t_p = tau_r tau_d/(tau_d - tau_r) ln(tau_d/tau_r); f = 1/g(t_p), so that one
 * event of weight w gives a conductance whose peak is exactly w.           */
double orc_syn_peak_factor(double tau_r, double tau_d, double *t_peak) {
    double tp = tau_r * tau_d / (tau_d - tau_r) * log(tau_d / tau_r);
    if (t_peak) *t_peak = tp;
    return 1.0 / (exp(-tp / tau_d) - exp(-tp / tau_r));
}

/* -------------------------------------------------------------- events -- */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the n-th output (n >= 1) of
 * the generator started at `seed` is mix(seed + n*gamma).  The event draw of
 * synapse gid at step k is output number n = gid*2^32 + k + 1.              */
uint64_t orc_event_hash(uint64_t seed, int64_t gid, int64_t k) {
    uint64_t n = ((uint64_t)gid << 32) + (uint64_t)k + 1u;
    uint64_t z = seed + n * UINT64_C(0x9E3779B97F4A7C15);
    z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);
    z = (z ^ (z >> 27)) * UINT64_C(0x94D049BB133111EB);
    return z ^ (z >> 31);
}

/* A synapse fires at a step with probability p = rate*dt (dt in ms): the
 * draw is compared with T = floor(p * 2^64).                                */
uint64_t orc_event_threshold(double rate_hz, double dt) {
    double p = rate_hz * dt * 1e-3;
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return UINT64_MAX;
    return (uint64_t)floor(p * 18446744073709551616.0);
}

/* ------------------------------------------------------------- current -- */
/* The calcium concentration a cahva or capump instance sees: its own pool,
 * or under shared_ca its node's.                                           */
static double ca_conc(const orc_globals *gl, const orc_nodes *nd, const orc_slot *s, int64_t i) {
    return (gl->shared_ca && nd && nd->cai) ? nd->cai[s->node[i]] : s->st[2][i];
}

/* Current of one instance at potential v with every STATE frozen:
 * density mechanisms in mA/cm2, the synapse in nA.                         */
static double instance_i(const orc_globals *gl, const orc_nodes *nd, const orc_slot *s, int64_t i, double v) {
    switch (s->kind) {
    case ORC_PAS:
        return s->par[0][i] * (v - s->par[1][i]);
    case ORC_HH: {
        double m = s->st[0][i], h = s->st[1][i], n = s->st[2][i];
        double gna = s->par[0][i] * m * m * m * h;
        double gk = s->par[1][i] * n * n * n * n;
        return gna * (v - gl->ena) + gk * (v - gl->ek) + s->par[2][i] * (v - s->par[3][i]);
    }
    case ORC_IH:
        return s->par[0][i] * s->st[0][i] * (v - gl->eh);
    case ORC_CAHVA:
    case ORC_CAPUMP:
    case ORC_CABUF: {
        double m = s->st[0][i], h = s->st[1][i];
        double eca = orc_nernst_ca(ca_conc(gl, nd, s, i), gl->cao, gl->celsius);
        return s->par[0][i] * m * m * h * (v - eca);
    }
    case ORC_KMARKOV:
        return s->par[0][i] * s->st[2][i] * (v - gl->ek);
    case ORC_SYN: {
        double ga = s->st[1][i] - s->st[0][i];
        double gn = s->st[3][i] - s->st[2][i];
        /* nS * mV = pA; 1e-3 converts to nA */
        return 1e-3 * (ga + gn * orc_mg_block(v, gl->mg)) * (v - gl->e_syn);
    }
    }
    return 0.0;
}

/* di/dv in closed form with every STATE frozen (section 5.2: the
 * conductance known from the AST instead of a run-time difference).  Ohmic
 * currents give their conductance products; the NMDA term also carries the
 * slope of the Mg block, B'(v) = 0.062 B (1 - B).                          */
static double instance_g(const orc_globals *gl, const orc_slot *s, int64_t i, double v) {
    switch (s->kind) {
    case ORC_PAS:
        return s->par[0][i];
    case ORC_HH: {
        double m = s->st[0][i], h = s->st[1][i], n = s->st[2][i];
        return s->par[0][i] * m * m * m * h + s->par[1][i] * n * n * n * n + s->par[2][i];
    }
    case ORC_IH:
        return s->par[0][i] * s->st[0][i];
    case ORC_CAHVA:
    case ORC_CAPUMP:
    case ORC_CABUF: {
        double m = s->st[0][i], h = s->st[1][i];
        return s->par[0][i] * m * m * h;
    }
    case ORC_KMARKOV:
        return s->par[0][i] * s->st[2][i];
    case ORC_SYN: {
        double ga = s->st[1][i] - s->st[0][i];
        double gn = s->st[3][i] - s->st[2][i];
        double B = orc_mg_block(v, gl->mg);
        return 1e-3 * (ga + gn * (B + (v - gl->e_syn) * 0.062 * B * (1.0 - B)));
    }
    }
    return 0.0;
}

void orc_instance_current(const orc_globals *gl, const orc_nodes *nd, const orc_slot *s, int64_t i,
                          double v, double *cur, double *cond) {
    double i0 = instance_i(gl, nd, s, i, v);
    *cur = i0;
    if (gl->analytic_conductance) {
        *cond = instance_g(gl, s, i, v);
    } else {
        double i1 = instance_i(gl, nd, s, i, v + gl->fd_dv);
        *cond = (i1 - i0) / gl->fd_dv;
    }
}

/* Sum of the magnitudes of the terms that make up instance_i, at v.        */
static double instance_terms(const orc_globals *gl, const orc_nodes *nd, const orc_slot *s, int64_t i, double v) {
    switch (s->kind) {
    case ORC_HH: {
        double m = s->st[0][i], h = s->st[1][i], n = s->st[2][i];
        double gna = s->par[0][i] * m * m * m * h;
        double gk = s->par[1][i] * n * n * n * n;
        return fabs(gna * (v - gl->ena)) + fabs(gk * (v - gl->ek)) + fabs(s->par[2][i] * (v - s->par[3][i]));
    }
    case ORC_SYN: {
        double ga = s->st[1][i] - s->st[0][i];
        double gn = s->st[3][i] - s->st[2][i];
        return 1e-3 * (fabs(ga) + fabs(gn * orc_mg_block(v, gl->mg))) * fabs(v - gl->e_syn);
    }
    default:
        return fabs(instance_i(gl, nd, s, i, v));
    }
}

void orc_node_scales(const orc_globals *gl, const orc_nodes *nd, const orc_slot *slots, int nslots,
                     double *terms, double *gsum, int32_t *count) {
    for (int64_t n = 0; n < nd->n_nodes; ++n) {
        terms[n] = 0.0;
        gsum[n] = 0.0;
        count[n] = 0;
    }
    for (int s = 0; s < nslots; ++s) {
        const orc_slot *sl = &slots[s];
        for (int64_t i = 0; i < sl->n; ++i) {
            int32_t ni = sl->node[i];
            double v = nd->v[ni], I0, g;
            double sc = sl->kind == ORC_SYN ? 1e2 / nd->area[ni] : 1.0;
            orc_instance_current(gl, nd, sl, i, v, &I0, &g);
            terms[ni] += sc * instance_terms(gl, nd, sl, i, v);
            gsum[ni] += fabs(sc * g);
            count[ni] += 1;
        }
    }
}

/* --------------------------------------------------------------- phases -- */
void orc_init(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots) {
    for (int s = 0; s < nslots; ++s) {
        orc_slot *sl = &slots[s];
        for (int64_t i = 0; i < sl->n; ++i) {
            double v = nd->v[sl->node[i]];
            double o[6];
            switch (sl->kind) {
            case ORC_HH:
                orc_hh_inf_tau(v, gl->celsius, o);
                sl->st[0][i] = o[0]; sl->st[1][i] = o[1]; sl->st[2][i] = o[2];
                break;
            case ORC_IH:
                orc_ih_inf_tau(v, o);
                sl->st[0][i] = o[0];
                break;
            case ORC_CAHVA:
            case ORC_CAPUMP:
            case ORC_CABUF:
                orc_cahva_inf_tau(v, o);
                sl->st[0][i] = o[0]; sl->st[1][i] = o[1]; sl->st[2][i] = gl->cai0;
                if (sl->kind == ORC_CABUF) sl->st[3][i] = orc_cabuf_bound(gl, gl->cai0);
                if (sl->ica) sl->ica[i] = 0.0;
                break;
            case ORC_KMARKOV: {
                orc_hh_inf_tau(v, gl->celsius, o);
                double n = o[2];
                sl->st[0][i] = (1.0 - n) * (1.0 - n);
                sl->st[1][i] = 2.0 * n * (1.0 - n);
                sl->st[2][i] = n * n;
                break;
            }
            case ORC_SYN:
                for (int j = 0; j < 4; ++j) sl->st[j][i] = 0.0;
                break;
            default:
                break;
            }
        }
    }
    if (nd->spikes)
        for (int64_t n = 0; n < nd->n_nodes; ++n) nd->spikes[n] = 0;
    if (nd->cai)
        for (int64_t n = 0; n < nd->n_nodes; ++n) nd->cai[n] = gl->cai0;
    if (nd->ica)
        for (int64_t n = 0; n < nd->n_nodes; ++n) nd->ica[n] = 0.0;
}

void orc_events(const orc_globals *gl, orc_slot *slots, int nslots, int64_t k, double dt) {
    uint64_t T = orc_event_threshold(gl->event_rate_hz, dt);
    double fa = orc_syn_peak_factor(gl->tau_r_ampa, gl->tau_d_ampa, NULL);
    double fn = orc_syn_peak_factor(gl->tau_r_nmda, gl->tau_d_nmda, NULL);
    for (int s = 0; s < nslots; ++s) {
        orc_slot *sl = &slots[s];
        if (sl->kind != ORC_SYN) continue;
        for (int64_t i = 0; i < sl->n; ++i) {
            int64_t gid = sl->gid ? sl->gid[i] : i;
            if (orc_event_hash(gl->event_seed, gid, k) < T) {
                double w = sl->par[0][i];
                sl->st[0][i] += w * fa;
                sl->st[1][i] += w * fa;
                sl->st[2][i] += w * fn;
                sl->st[3][i] += w * fn;
            }
        }
    }
}

void orc_cur(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots) {
    const int shared = gl->shared_ca && nd->cai && nd->ica;
    for (int64_t n = 0; n < nd->n_nodes; ++n) { nd->rhs[n] = 0.0; nd->d[n] = 0.0; }
    if (shared)
        for (int64_t n = 0; n < nd->n_nodes; ++n) nd->ica[n] = 0.0;
    for (int s = 0; s < nslots; ++s) {
        orc_slot *sl = &slots[s];
        for (int64_t i = 0; i < sl->n; ++i) {
            int32_t ni = sl->node[i];
            double I0, g;
            orc_instance_current(gl, nd, sl, i, nd->v[ni], &I0, &g);
            if (sl->kind == ORC_CAHVA || sl->kind == ORC_CAPUMP || sl->kind == ORC_CABUF) {
                if (sl->ica) sl->ica[i] = I0;
                if (shared) nd->ica[ni] += I0;   /* the node's calcium current */
            }
            if (sl->kind == ORC_SYN) {
                /* nA/um2 -> mA/cm2 and uS/um2 -> S/cm2: both a factor 100 */
                double sc = 1e2 / nd->area[ni];
                nd->rhs[ni] -= sc * I0;
                nd->d[ni] += sc * g;
            } else {
                nd->rhs[ni] -= I0;
                nd->d[ni] += g;
            }
        }
    }
}

void orc_vclamp(orc_nodes *nd, double t) {
    for (int64_t n = 0; n < nd->n_nodes; ++n)
        nd->v[n] = nd->clamp_off[n] +
                   nd->clamp_amp[n] * sin(2.0 * ORC_PI * nd->clamp_freq[n] * t * 1e-3 + nd->clamp_phase[n]);
}

/* Backward Euler for an isolated compartment, linearised in v:
 * 1e-3*cm*(v_new - v)/dt = rhs - d*(v_new - v).                              */
void orc_visolated(const orc_globals *gl, orc_nodes *nd, double dt) {
    for (int64_t n = 0; n < nd->n_nodes; ++n) {
        double v0 = nd->v[n];
        double v1 = v0 + nd->rhs[n] / (1e-3 * nd->cm[n] / dt + nd->d[n]);
        if (nd->spikes && v0 < gl->vthresh && v1 >= gl->vthresh) nd->spikes[n] += 1;
        nd->v[n] = v1;
    }
}

/* Hines (1984) elimination on the tree matrix: node n's row holds
 * D_n = 1e-3 cm/dt + d_n + sum of its couplings, -k_{n,p} towards its parent
 * p and -k_{n,c} towards each child c.  Eliminating children into parents
 * from the highest index down leaves a triangular system solved from the
 * roots up.  parent[n] < n makes that order valid.                         */
void orc_vcable(const orc_globals *gl, orc_nodes *nd, double dt) {
    int64_t N = nd->n_nodes;
    double *D = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *R = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int64_t n = 0; n < N; ++n) {
        D[n] = 1e-3 * nd->cm[n] / dt + nd->d[n];
        R[n] = nd->rhs[n];
    }
    for (int64_t n = 0; n < N; ++n) {
        int32_t p = nd->parent[n];
        if (p < 0) continue;
        double kn = 1e2 * nd->g_axial[n] / nd->area[n];   /* row n, towards p */
        double kp = 1e2 * nd->g_axial[n] / nd->area[p];   /* row p, towards n */
        D[n] += kn;
        D[p] += kp;
        R[n] += kn * (nd->v[p] - nd->v[n]);
        R[p] += kp * (nd->v[n] - nd->v[p]);
    }
    for (int64_t n = N - 1; n >= 0; --n) {
        int32_t p = nd->parent[n];
        if (p < 0) continue;
        double kn = 1e2 * nd->g_axial[n] / nd->area[n];
        double kp = 1e2 * nd->g_axial[n] / nd->area[p];
        double f = -kp / D[n];           /* row p's entry in column n over D_n */
        D[p] -= f * -kn;
        R[p] -= f * R[n];
    }
    for (int64_t n = 0; n < N; ++n) {
        int32_t p = nd->parent[n];
        double dv = p < 0 ? R[n] / D[n] : (R[n] - (-(1e2 * nd->g_axial[n] / nd->area[n])) * R[p]) / D[n];
        R[n] = dv;   /* R now holds dv, parents before children */
    }
    for (int64_t n = 0; n < N; ++n) {
        double v0 = nd->v[n], v1 = v0 + R[n];
        if (nd->spikes && v0 < gl->vthresh && v1 >= gl->vthresh) nd->spikes[n] += 1;
        nd->v[n] = v1;
    }
    free(D);
    free(R);
}

/* cnexp: x' = (x_inf - x)/tau with x_inf and tau frozen over the step has the
 * exact solution x(t+dt) = x_inf + (x - x_inf) exp(-dt/tau) (section 5.2).
 * With pade_cnexp the factor exp(-y) is the (1,1) Pade approximant
 * (1 - y/2)/(1 + y/2), y = dt/tau (section 5.2, optional replacement).     */
static double decay_factor(const orc_globals *gl, double dt, double tau) {
    double y = dt / tau;
    if (gl->pade_cnexp) return (1.0 - y / 2.0) / (1.0 + y / 2.0);
    return exp(-y);
}

static double cnexp(const orc_globals *gl, double x, double xinf, double tau, double dt) {
    return xinf + (x - xinf) * decay_factor(gl, dt, tau);
}

void orc_state(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots, double dt) {
    double kappa = orc_ca_kappa(gl->ca_gamma, gl->ca_depth);
    const int shared = gl->shared_ca && nd->cai && nd->ica;
    for (int s = 0; s < nslots; ++s) {
        orc_slot *sl = &slots[s];
        for (int64_t i = 0; i < sl->n; ++i) {
            double v = nd->v[sl->node[i]];
            double o[6];
            switch (sl->kind) {
            case ORC_HH:
                orc_hh_inf_tau(v, gl->celsius, o);
                sl->st[0][i] = cnexp(gl, sl->st[0][i], o[0], o[3], dt);
                sl->st[1][i] = cnexp(gl, sl->st[1][i], o[1], o[4], dt);
                sl->st[2][i] = cnexp(gl, sl->st[2][i], o[2], o[5], dt);
                break;
            case ORC_IH:
                orc_ih_inf_tau(v, o);
                sl->st[0][i] = cnexp(gl, sl->st[0][i], o[0], o[1], dt);
                break;
            case ORC_CAHVA: {
                orc_cahva_inf_tau(v, o);
                sl->st[0][i] = cnexp(gl, sl->st[0][i], o[0], o[2], dt);
                sl->st[1][i] = cnexp(gl, sl->st[1][i], o[1], o[3], dt);
                /* linear in cai with ica held at its stored value:
                 * cai_inf = cai0 - kappa*tau_ca*ica, time constant tau_ca   */
                if (!shared) {
                    double cinf = gl->cai0 - kappa * gl->tau_ca * sl->ica[i];
                    sl->st[2][i] = cnexp(gl, sl->st[2][i], cinf, gl->tau_ca, dt);
                }
                break;
            }
            case ORC_CAPUMP: {
                orc_cahva_inf_tau(v, o);
                sl->st[0][i] = cnexp(gl, sl->st[0][i], o[0], o[2], dt);
                sl->st[1][i] = cnexp(gl, sl->st[1][i], o[1], o[3], dt);
                if (!shared) orc_capump_step(gl, sl->ica[i], dt, &sl->st[2][i], gl->newton_iters);
                break;
            }
            case ORC_CABUF: {
                orc_cahva_inf_tau(v, o);
                sl->st[0][i] = cnexp(gl, sl->st[0][i], o[0], o[2], dt);
                sl->st[1][i] = cnexp(gl, sl->st[1][i], o[1], o[3], dt);
                if (!shared)
                    orc_cabuf_step(gl, sl->ica[i], dt, &sl->st[2][i], &sl->st[3][i], gl->newton_iters);
                break;
            }
            case ORC_KMARKOV: {
                double x[3] = {sl->st[0][i], sl->st[1][i], sl->st[2][i]};
                orc_kmarkov_step(v, gl->celsius, dt, x);
                sl->st[0][i] = x[0]; sl->st[1][i] = x[1]; sl->st[2][i] = x[2];
                break;
            }
            case ORC_SYN:
                sl->st[0][i] *= decay_factor(gl, dt, gl->tau_r_ampa);
                sl->st[1][i] *= decay_factor(gl, dt, gl->tau_d_ampa);
                sl->st[2][i] *= decay_factor(gl, dt, gl->tau_r_nmda);
                sl->st[3][i] *= decay_factor(gl, dt, gl->tau_d_nmda);
                break;
            default:
                break;
            }
        }
    }
    /* one pool per node, driven by the node's total calcium current: the same
     * linear law as a cahva instance's own pool                             */
    if (shared)
        for (int64_t n = 0; n < nd->n_nodes; ++n) {
            double cinf = gl->cai0 - kappa * gl->tau_ca * nd->ica[n];
            nd->cai[n] = cnexp(gl, nd->cai[n], cinf, gl->tau_ca, dt);
        }
}

int orc_run(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots,
            int64_t k0, int64_t nsteps, double dt, int vmode) {
    if (!gl || !nd || (nslots > 0 && !slots) || nsteps < 0 || !(dt > 0.0)) return -1;
    if (vmode == ORC_V_CLAMP) orc_vclamp(nd, (double)k0 * dt);
    for (int64_t k = k0; k < k0 + nsteps; ++k) {
        orc_events(gl, slots, nslots, k, dt);
        orc_cur(gl, nd, slots, nslots);
        if (vmode == ORC_V_CLAMP) orc_vclamp(nd, (double)(k + 1) * dt);
        else if (vmode == ORC_V_ISOLATED) orc_visolated(gl, nd, dt);
        else if (vmode == ORC_V_CABLE) orc_vcable(gl, nd, dt);
        orc_state(gl, nd, slots, nslots, dt);
    }
    return 0;
}
