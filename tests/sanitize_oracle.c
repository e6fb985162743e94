/*
 * sanitize_oracle.c -- drives every phase of the CPU oracle on random meshes
 * under AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py
 * builds and runs it).  Every array is allocated at its exact size, so a read
 * or write one element past any of them is reported.
 *
 * Covered: all eight mechanism kinds with many-to-one node indices, the four
 * voltage modes (random branched trees for the cable mode), the calcium pool
 * per instance and per node, the closed-form conductance and Pade variants.
 * Exit status 0 when every result is finite, 1 otherwise (a sanitizer report
 * aborts with its own status first).
 */
#include "mech_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}
static double uni(double lo, double hi) { return lo + (hi - lo) * (double)(next_u64() >> 11) / 9007199254740992.0; }
static int below(int n) { return (int)(next_u64() % (uint64_t)n); }

static double *dalloc(int64_t n, double lo, double hi) {
    double *a = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) a[i] = uni(lo, hi);
    return a;
}

#define NK 8
static const int kStates[NK] = {0, 3, 1, 3, 4, 3, 3, 4};
static const int kParams[NK] = {2, 4, 1, 1, 1, 1, 1, 1};

static int finite_all(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run_case(int n_nodes, int vmode, int shared, int analytic, int pade, int64_t nsteps) {
    orc_globals gl = {6.3, 50.0, -77.0, -45.0, 2.0, 5e-5, 80.0, 0.05, 0.1, 0.0, 1.0, 0.2, 1.7, 0.29, 43.0,
                      400.0, -20.0, 1e-3, 12345u, analytic, pade, 1e-4, 1e-3, 4, shared, 0.05, 100.0, 0.1};
    orc_nodes nd;
    nd.n_nodes = n_nodes;
    nd.v = dalloc(n_nodes, -80.0, -50.0);
    nd.rhs = dalloc(n_nodes, 0.0, 0.0);
    nd.d = dalloc(n_nodes, 0.0, 0.0);
    double *area = dalloc(n_nodes, 100.0, 1000.0);
    double *cm = dalloc(n_nodes, 0.8, 1.2);
    double *off = dalloc(n_nodes, -80.0, 20.0), *amp = dalloc(n_nodes, 0.0, 40.0);
    double *freq = dalloc(n_nodes, 5.0, 50.0), *phase = dalloc(n_nodes, 0.0, 6.28);
    nd.area = area;
    nd.cm = cm;
    nd.clamp_off = off;
    nd.clamp_amp = amp;
    nd.clamp_freq = freq;
    nd.clamp_phase = phase;
    nd.spikes = malloc(sizeof(int32_t) * (size_t)n_nodes);
    /* cells of random size, each a random tree in Hines order */
    int32_t *parent = malloc(sizeof(int32_t) * (size_t)n_nodes);
    double *g_axial = dalloc(n_nodes, 0.01, 0.5);
    for (int n = 0; n < n_nodes;) {
        int size = 1 + below(40);
        if (n + size > n_nodes) size = n_nodes - n;
        parent[n] = -1;
        g_axial[n] = 0.0;
        for (int j = 1; j < size; ++j) parent[n + j] = n + below(j);
        n += size;
    }
    nd.parent = parent;
    nd.g_axial = g_axial;
    nd.cai = dalloc(n_nodes, 0.0, 0.0);
    nd.ica = dalloc(n_nodes, 0.0, 0.0);

    orc_slot slots[NK];
    int32_t *nodes[NK];
    int64_t *gids[NK];
    for (int k = 0; k < NK; ++k) {
        orc_slot *s = &slots[k];
        s->kind = k;
        s->n = below(3 * n_nodes + 1);
        nodes[k] = malloc(sizeof(int32_t) * (size_t)(s->n > 0 ? s->n : 1));
        for (int64_t i = 0; i < s->n; ++i) nodes[k][i] = below(n_nodes);
        s->node = nodes[k];
        gids[k] = NULL;
        if (k == ORC_SYN) {
            gids[k] = malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
            for (int64_t i = 0; i < s->n; ++i) gids[k][i] = (int64_t)(next_u64() >> 40);
        }
        s->gid = gids[k];
        double *par[4] = {NULL, NULL, NULL, NULL};
        for (int j = 0; j < kParams[k]; ++j) par[j] = dalloc(s->n, 1e-5, 1e-3);
        if (k == ORC_PAS) for (int64_t i = 0; i < s->n; ++i) par[1][i] = uni(-75.0, -60.0);
        if (k == ORC_HH) for (int64_t i = 0; i < s->n; ++i) par[3][i] = uni(-60.0, -50.0);
        if (k == ORC_SYN) for (int64_t i = 0; i < s->n; ++i) par[0][i] = uni(0.5, 3.0);
        for (int j = 0; j < 4; ++j) {
            s->st[j] = j < kStates[k] ? dalloc(s->n, 0.0, 0.0) : NULL;
            s->par[j] = par[j];
        }
        s->ica = (k == ORC_CAHVA || k == ORC_CAPUMP || k == ORC_CABUF) ? dalloc(s->n, 0.0, 0.0) : NULL;
    }

    orc_init(&gl, &nd, slots, NK);
    int ok = orc_run(&gl, &nd, slots, NK, 0, nsteps, 0.025, vmode) == 0;
    double I, G;
    for (int k = 0; k < NK; ++k)
        if (slots[k].n > 0) orc_instance_current(&gl, &nd, &slots[k], slots[k].n - 1, -30.0, &I, &G);
    ok = ok && finite_all(nd.v, n_nodes) && finite_all(nd.rhs, n_nodes) && finite_all(nd.d, n_nodes) &&
         finite_all(nd.cai, n_nodes);
    for (int k = 0; k < NK; ++k)
        for (int j = 0; j < kStates[k]; ++j) ok = ok && finite_all(slots[k].st[j], slots[k].n);

    for (int k = 0; k < NK; ++k) {
        for (int j = 0; j < 4; ++j) {
            free(slots[k].st[j]);
            free((void *)slots[k].par[j]);
        }
        free(slots[k].ica);
        free(nodes[k]);
        free(gids[k]);
    }
    free(nd.v); free(nd.rhs); free(nd.d); free(area); free(cm);
    free(off); free(amp); free(freq); free(phase);
    free(nd.spikes); free(parent); free(g_axial); free(nd.cai); free(nd.ica);
    return ok;
}

int main(void) {
    int ok = 1, cases = 0;
    for (int vmode = ORC_V_EXTERNAL; vmode <= ORC_V_CABLE; ++vmode)
        for (int shared = 0; shared <= 1; ++shared)
            for (int variant = 0; variant < 3; ++variant)
                for (int size = 1; size <= 257; size += 64) {
                    ok &= run_case(size, vmode, shared, variant == 1, variant == 2, 30);
                    ++cases;
                }
    /* the single-point functions at their removable singularities */
    double o[9];
    orc_hh_inf_tau(-40.0, 6.3, o);
    orc_hh_inf_tau(-55.0, 6.3, o);
    orc_hh_rates(-40.0, o);
    orc_ih_inf_tau(-90.0, o);
    orc_cahva_inf_tau(-27.0, o);
    orc_kmarkov_matrix(-40.0, 6.3, 0.025, o);
    ok &= isfinite(orc_syn_peak_factor(0.2, 1.7, NULL)) && isfinite(orc_nernst_ca(5e-5, 2.0, 6.3));
    printf("%d cases, %s\n", cases, ok ? "all finite" : "NON-FINITE RESULT");
    return ok ? 0 : 1;
}
