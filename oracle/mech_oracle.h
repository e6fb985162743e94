/*
 * mech_oracle.h -- plain FP64 CPU oracle for the per-timestep mechanism kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (paper: section 3, NMODL blocks; section 5.2, cnexp; section
 * 5.2 last paragraph, numerically approximated conductance; section 8 and
 * Table 3, the State Update / Current Update / Other split of a timestep):
 *
 *   one timestep k (t_k = k*dt, never a running sum):
 *     1. events   : every synapse whose counter-based draw H(seed,gid,k) lies
 *                   below T = floor(rate*dt*1e-3 * 2^64) receives w*f on both
 *                   rise and decay states of both receptors;
 *     2. cur      : rhs = d = 0, then for every slot in order and every instance
 *                   in index order: I0 = i(v), I1 = i(v+dv), g = (I1-I0)/dv,
 *                   rhs[node] -= s*I0, d[node] += s*g  (s = 1 for density
 *                   mechanisms, s = 100/area for point processes); under
 *                   shared_ca the calcium currents are also summed per node;
 *     3. voltage  : CLAMP    v = off + amp*sin(2*pi*freq*t_{k+1}*1e-3 + phase)
 *                   ISOLATED v += rhs/(1e-3*cm/dt + d), count upward crossings
 *                   of vthresh
 *                   CABLE    backward Euler of the cable equation on the cell
 *                   trees (Hines elimination), crossings counted as ISOLATED
 *                   EXTERNAL v unchanged;
 *     4. state    : update of every STATE at the new v (cnexp, or the implicit
 *                   solves of kmarkov and capump), then under shared_ca each
 *                   node's calcium pool.
 *
 * Units: mV, ms, mA/cm2 and S/cm2 (density), nA and uS (point process),
 * um2, uF/cm2, mM, degC; synaptic weights and states in nS.
 *
 * Parity pins: every function here is pinned in tests/ against closed forms,
 * invariants, published values or brute force.  The Ih and Ca-HVA rate
 * constants are this project's own synthetic definitions; beyond the closed
 * forms and invariants they are pinned to nothing external ("parity unpinned"
 * for their constants, see the test module docstrings).
 */
#ifndef MECH_ORACLE_H
#define MECH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PAS = 0, ORC_HH = 1, ORC_IH = 2, ORC_CAHVA = 3, ORC_SYN = 4, ORC_KMARKOV = 5, ORC_CAPUMP = 6,
       ORC_CABUF = 7 };
enum { ORC_V_EXTERNAL = 0, ORC_V_CLAMP = 1, ORC_V_ISOLATED = 2, ORC_V_CABLE = 3 };

/* One mechanism type ("slot") and its instances, in the caller's order.
 *   st : STATE arrays     hh: m,h,n   ih: m   cahva: m,h,cai   syn: Aa,Ba,An,Bn
 *                         kmarkov: C1,C2,O   capump: m,h,cai
 *                         cabuf: m,h,cai,cab
 *   par: RANGE parameters hh: gnabar,gkbar,gl,el   pas: g,e   ih: gbar
 *                         cahva: gbar   syn: weight (nS)   kmarkov: gbar
 *                         capump: gbar   cabuf: gbar
 *   ica: Ca-HVA calcium current written by cur and read by state (mA/cm2)
 *   gid: synapse event-stream id (NULL: the instance index is used)        */
typedef struct {
    int32_t kind;
    int64_t n;
    const int32_t *node;
    const int64_t *gid;
    double *st[4];
    const double *par[4];
    double *ica;
} orc_slot;

typedef struct {
    double celsius;                 /* degC                                  */
    double ena, ek, eh;             /* mV                                    */
    double cao, cai0, tau_ca;       /* mM, mM, ms                            */
    double ca_gamma, ca_depth;      /* free fraction, shell depth (um)       */
    double e_syn, mg;               /* mV, mM                                */
    double tau_r_ampa, tau_d_ampa;  /* ms                                    */
    double tau_r_nmda, tau_d_nmda;  /* ms                                    */
    double event_rate_hz;           /* Hz                                    */
    double vthresh;                 /* mV                                    */
    double fd_dv;                   /* mV                                    */
    uint64_t event_seed;
    /* section 5.2 variants, both off by default:
     * analytic_conductance: g = di/dv in closed form instead of the finite
     *   difference (the CONDUCTANCE statement the framework generates);
     * pade_cnexp: the cnexp factor exp(-x), x = dt/tau, is replaced by its
     *   (1,1) Pade approximant (1 - x/2)/(1 + x/2).                          */
    int32_t analytic_conductance;
    int32_t pade_cnexp;
    /* capump: Michaelis-Menten pump of maximal rate vmax (mM/ms) and
     * half-activation kp (mM), balanced at cai0; newton_iters Newton steps
     * solve its implicit Euler equation (section 5.2, derivimplicit).        */
    double pump_vmax, pump_kp;
    int32_t newton_iters;
    /* shared_ca: calcium is a per-node ion (USEION ca, section 3): every
     * cahva and capump instance reads its node's cai and adds its ica to the
     * node's total, and one pool per node relaxes by the linear pool law
     * from that total (the instances' own pools are not used).              */
    int32_t shared_ca;
    /* cabuf: total buffer (mM), binding rate (1/(mM ms)) and unbinding rate
     * (1/ms) of the calcium buffer                                          */
    double buf_total, buf_kon, buf_koff;
} orc_globals;

typedef struct {
    int64_t n_nodes;
    double *v, *rhs, *d;
    const double *area;             /* um2, NULL if no point process        */
    const double *cm;               /* uF/cm2, ISOLATED mode only            */
    const double *clamp_off, *clamp_amp, *clamp_freq, *clamp_phase;
    int32_t *spikes;                /* ISOLATED and CABLE modes              */
    /* CABLE mode (section 8, Table 3 "Other": the tree solve between the
     * current and the state update): parent[n] < n is node n's parent in its
     * cell (-1 for a root), g_axial[n] the conductance (uS) of the segment
     * between node n and its parent.                                        */
    const int32_t *parent;
    const double *g_axial;
    /* shared_ca: the node's calcium concentration (mM) and total calcium
     * current density (mA/cm2) of the last current update.                  */
    double *cai, *ica;
} orc_nodes;

/* ---- single-point functions (used by the pins) ----------------------- */
/* out = {m_inf, h_inf, n_inf, tau_m, tau_h, tau_n}                         */
void orc_hh_inf_tau(double v, double celsius, double *out6);
/* out = {alpha_m, beta_m, alpha_h, beta_h, alpha_n, beta_n} (1/ms, q10 = 1) */
void orc_hh_rates(double v, double *out6);
void orc_ih_inf_tau(double v, double *out2);                 /* m_inf, tau_m */
void orc_cahva_inf_tau(double v, double *out4);   /* m_inf, h_inf, tau_m, tau_h */
/* kmarkov: the 3x3 implicit Euler matrix M = I - dt A(v) (row-major) and
 * one implicit Euler step x <- M^{-1} x by Gaussian elimination with
 * partial pivoting (section 5.2, sparse method).                           */
void orc_kmarkov_matrix(double v, double celsius, double dt, double *M9);
void orc_kmarkov_step(double v, double celsius, double dt, double *x3);
/* capump: one implicit Euler step of the pool, cai <- root of
 * c - cai - dt F(c) = 0 with F(c) = -kappa ica - vmax (c/(c+kp) -
 * cai0/(cai0+kp)), by `iters` Newton steps from c = cai; returns the
 * residual of the last iterate.                                           */
double orc_capump_step(const orc_globals *gl, double ica, double dt, double *cai, int iters);
/* one implicit Euler step of the cabuf pool (free cai, bound cab), `iters`
 * Newton steps on the 2x2 system; returns the max-norm residual            */
double orc_cabuf_step(const orc_globals *gl, double ica, double dt, double *cai, double *cab, int iters);
double orc_cabuf_bound(const orc_globals *gl, double c);        /* mM        */
double orc_mg_block(double v, double mg);
double orc_syn_peak_factor(double tau_r, double tau_d, double *t_peak);
double orc_nernst_ca(double cai, double cao, double celsius);     /* mV      */
double orc_ca_kappa(double gamma, double depth);   /* mM/ms per mA/cm2      */
uint64_t orc_event_hash(uint64_t seed, int64_t gid, int64_t k);
uint64_t orc_event_threshold(double rate_hz, double dt);
/* current of one instance at v with frozen states: *i = I(v), *g = di/dv
 * (finite difference, or closed form under analytic_conductance); nd gives
 * the node's cai under shared_ca and may be NULL otherwise                  */
void orc_instance_current(const orc_globals *gl, const orc_nodes *nd, const orc_slot *s, int64_t i,
                          double v, double *cur, double *cond);

/* Per-node scales of the rounding error of the current update, for the
 * parity tolerances (not part of the method): at each instance's node v,
 * terms[n] += |s| T_i where T_i is the sum of the magnitudes of the terms
 * added into the instance's current (hh: its three ionic currents; the
 * synapse: its two receptor currents; the other kinds: |I|), gsum[n] +=
 * |s g_i| and count[n] += 1, with s = 100/area for the synapse and 1
 * otherwise.  The outputs are overwritten.                                  */
void orc_node_scales(const orc_globals *gl, const orc_nodes *nd, const orc_slot *slots, int nslots,
                     double *terms, double *gsum, int32_t *count);

/* ---- phases and the full step loop ------------------------------------ */
void orc_init(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots);
void orc_events(const orc_globals *gl, orc_slot *slots, int nslots, int64_t k, double dt);
void orc_cur(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots);
void orc_vclamp(orc_nodes *nd, double t);
void orc_visolated(const orc_globals *gl, orc_nodes *nd, double dt);
/* Backward Euler of the cable equation linearised in v:
 * (1e-3 cm/dt + d_n) dv_n + sum_j k_nj (dv_n - dv_j) = rhs_n + sum_j k_nj (v_j - v_n)
 * with k_nj = 100 g_nj / area_n (S/cm2) over the tree neighbours j of n,
 * solved by Hines' elimination (leaves to root, then root to leaves), then
 * v += dv and spike counting as in ISOLATED mode.                         */
void orc_vcable(const orc_globals *gl, orc_nodes *nd, double dt);
void orc_state(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots, double dt);
/* runs steps k0 .. k0+nsteps-1; in CLAMP mode v is first set to the clamp
 * value at t_{k0}.  Returns 0, or -1 on a bad argument.                   */
int orc_run(const orc_globals *gl, orc_nodes *nd, orc_slot *slots, int nslots,
            int64_t k0, int64_t nsteps, double dt, int vmode);

#ifdef __cplusplus
}
#endif
#endif
