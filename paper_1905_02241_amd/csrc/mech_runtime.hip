// mech_runtime.hip -- host side of libmech.so: the C ABI of include/mech.h.
//
// Responsibilities: argument validation, stable node sort of every mechanism
// type, carving of the caller's device buffer into 256-byte aligned SoA
// arrays, the tile table of the fused path, the launch sequences of the
// plain, batched (replayed from HIP graphs) and time-fused paths, the cut of
// cell trees into units for the cable solve, the launch-shape autotuners,
// host copies of STATEs in the caller's order, and roctx trace ranges.
#include "mech.h"
#include "mech_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace mech;

// Device memory of the contexts made by mech_alloc_static (see the static
// device area below): 64 MiB on every device the library runs on.
constexpr size_t kStaticBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticBytes];

namespace {

// ----------------------------------------------------------- type table --
struct VarDesc {
    const char *name;
    bool is_double;  // stored as double in both precisions (else the state type: every RANGE
                     // parameter read each step is, the driving force is still formed in FP64)
};
struct KindDesc {
    const char *name;
    bool point_process;
    int n_state;
    const char *state[kMaxStates];
    int n_param;
    VarDesc param[kMaxParams];
    double defaults[kMaxParams];
};

const KindDesc kKinds[8] = {
    {"pas", false, 0, {}, 2, {{"g", false}, {"e", false}}, {1e-3, -70.0}},
    {"hh", false, 3, {"m", "h", "n"}, 4,
     {{"gnabar", false}, {"gkbar", false}, {"gl", false}, {"el", false}}, {0.12, 0.036, 0.0003, -54.3}},
    {"ih", false, 1, {"m"}, 1, {{"gbar", false}}, {1e-4}},
    {"cahva", false, 3, {"m", "h", "cai"}, 1, {{"gbar", false}}, {5e-5}},
    {"syn", true, 4, {"A_ampa", "B_ampa", "A_nmda", "B_nmda"}, 1, {{"weight", true}}, {1.0}},
    {"kmarkov", false, 3, {"C1", "C2", "O"}, 1, {{"gbar", false}}, {0.01}},
    {"capump", false, 3, {"m", "h", "cai"}, 1, {{"gbar", false}}, {5e-5}},
    {"cabuf", false, 4, {"m", "h", "cai", "cab"}, 1, {{"gbar", false}}, {5e-5}},
};

struct Globals {
    double celsius = 6.3, ena = 50.0, ek = -77.0, eh = -45.0;
    double cao = 2.0, cai0 = 5e-5, tau_ca = 80.0, ca_gamma = 0.05, ca_depth = 0.1;
    double e_syn = 0.0, mg = 1.0;
    double tau_r_ampa = 0.2, tau_d_ampa = 1.7, tau_r_nmda = 0.29, tau_d_nmda = 43.0;
    double event_rate_hz = 5.0, vthresh = -20.0, fd_dv = 1e-3;
    uint64_t event_seed = 0;
    int analytic_conductance = 0;   // closed-form di/dv instead of the finite difference
    int pade_cnexp = 0;             // (1,1) Pade approximant of the cnexp exponential
    double pump_vmax = 1e-4, pump_kp = 1e-3;
    double buf_total = 0.05, buf_kon = 100.0, buf_koff = 0.1;
    int newton_iters = 4;
    int shared_ca = 0;              // calcium as a per-node ion
};

struct SlotHost {
    int kind = 0;
    int64_t n = 0, np = 0;
    bool identity = false;
    bool perm_identity = true;
    std::vector<int32_t> perm;     // internal -> caller index (empty when identity)
    std::vector<int32_t> ni;       // node index, internal (sorted) order
    size_t off_ni = 0, off_gid = 0, off_ica = 0;
    size_t off_carry = 0;          // plain path: per wave, a node (int) then three doubles
    size_t off_st[kMaxStates] = {}, off_par[kMaxParams] = {};
    bool has_gid = false, has_ica = false;
};

// Cell trees of the cable mode, cut into units on the host at
// mech_bind_cable (the unit kinds and positions are described with CableDev).
struct CableHost {
    std::vector<int32_t> parent, pos_node, pos_par, pos_src, elim_n, elim_p, elim_ptr, unit_pos, unit_elim,
        unit_mode, list_up, list_top, list_top_g, list_down, pos_pnode, elim_run;
    int lds_max = 0;
};

// Validates Hines order and contiguous cells, then cuts the trees into units
// of at most `cap` positions (a trunk may exceed it) and writes each unit's
// edge records bucketed by the child's height.  Returns "" on success.
std::string build_cable(int64_t N, const int32_t *parent, int cap, CableHost &h) {
    h = CableHost();
    if (cap < 1) cap = 1;
    std::vector<int32_t> first;
    for (int64_t n = 0; n < N; ++n) {
        const int32_t p = parent[n];
        if (p < -1 || p >= n) return "parent[n] must be -1 or a node index below n (Hines order)";
        if (p < 0) first.push_back((int32_t)n);
        else if (first.empty() || p < first.back())
            return "every cell must be a contiguous node range starting at its root";
    }
    if (N > 0 && (first.empty() || first[0] != 0)) return "node 0 must be a root";
    const int n_cells = (int)first.size();
    first.push_back((int32_t)N);
    h.parent.assign(parent, parent + N);
    std::vector<int32_t> sub(N, 1), ht(N, 0);
    for (int64_t n = N - 1; n >= 0; --n)
        if (parent[n] >= 0) {
            sub[parent[n]] += sub[n];
            ht[parent[n]] = std::max(ht[parent[n]], ht[n] + 1);
        }
    std::vector<int32_t> pos(N, -1), th(N, 0), levels;
    h.unit_pos.push_back(0);
    h.elim_ptr.push_back(0);
    struct Rec { int32_t h, n, p; };
    // closes the unit whose positions were placed last; recs are (height,
    // child position, parent position), a root paired with itself
    auto add_unit = [&](int mode, std::vector<Rec> &recs, int nlev) {
        const int u = (int)h.unit_mode.size();
        h.unit_mode.push_back(mode);
        h.unit_pos.push_back((int32_t)h.pos_node.size());
        h.unit_elim.push_back((int32_t)h.elim_ptr.size() - 1);
        // by height, and within a height by parent, so that a parent's
        // children of one height form a run that one thread folds in order
        std::stable_sort(recs.begin(), recs.end(),
                         [](const Rec &x, const Rec &y) { return x.h != y.h ? x.h < y.h : x.p < y.p; });
        size_t k = 0;
        for (int L = 0; L < nlev; ++L) {
            for (; k < recs.size() && recs[k].h == L; ++k) {
                h.elim_n.push_back(recs[k].n);
                h.elim_p.push_back(recs[k].p);
                // the head of a parent's run of this height carries the run's
                // length (at most kCableRunMax, longer runs are followed by
                // parent); the others 0
                int run = 0;
                if (k == 0 || recs[k - 1].h != L || recs[k - 1].p != recs[k].p)
                    while (k + run < recs.size() && recs[k + run].h == L && recs[k + run].p == recs[k].p &&
                           run < kCableRunMax)
                        ++run;
                h.elim_run.push_back(run);
            }
            h.elim_ptr.push_back((int32_t)h.elim_n.size());
        }
        levels.push_back(nlev);
        const int size = h.unit_pos[u + 1] - h.unit_pos[u];
        if (mode != kUnitTop || size <= cap) h.lds_max = std::max(h.lds_max, size);
        if (mode == kUnitFull || mode == kUnitPiece) h.list_up.push_back(u);
        if (mode == kUnitFull || mode == kUnitPiece) h.list_down.push_back(u);
        if (mode == kUnitTop) (size <= cap ? h.list_top : h.list_top_g).push_back(u);
    };
    auto place = [&](int32_t n, int32_t par_pos, int32_t src) {
        const int32_t i = (int32_t)h.pos_node.size();
        h.pos_node.push_back(n);
        h.pos_pnode.push_back(parent[n]);
        h.pos_par.push_back(par_pos);
        h.pos_src.push_back(src);
        return i;
    };

    // whole cells that fit, packed into forests of up to `pack` nodes so that
    // many small cells do not each take a workgroup
    int64_t fit_nodes = 0;
    for (int c = 0; c < n_cells; ++c)
        if (first[c + 1] - first[c] <= cap) fit_nodes += first[c + 1] - first[c];
    const int pack = (int)std::min<int64_t>(cap, std::max<int64_t>(1024, (fit_nodes + 511) / 512));
    std::vector<Rec> recs;
    int nlev = 0, cur = 0;
    auto close_full = [&]() {
        // every root's own record goes to the unit's top height
        for (Rec &r : recs)
            if (r.h < 0) r.h = nlev - 1;
        if (cur > 0) add_unit(kUnitFull, recs, nlev);
        recs.clear();
        nlev = 0;
        cur = 0;
    };
    for (int c = 0; c < n_cells; ++c) {
        const int32_t a = first[c], b = first[c + 1];
        if (b - a > cap) continue;
        if (cur + (b - a) > pack) close_full();
        for (int32_t n = a; n < b; ++n) {
            const int32_t p = parent[n];
            pos[n] = place(n, p >= 0 ? pos[p] : -1, -1);
            recs.push_back({p >= 0 ? ht[n] : -1, pos[n], p >= 0 ? pos[p] : pos[n]});
        }
        nlev = std::max(nlev, ht[a] + 1);
        cur += b - a;
    }
    close_full();

    // cells too large: maximal subtrees that fit become pieces, packed into
    // forests; the trunk (subtree larger than cap) is one unit
    for (int c = 0; c < n_cells; ++c) {
        const int32_t a = first[c], b = first[c + 1];
        if (b - a <= cap) continue;
        std::vector<int32_t> pid(b - a, -1), roots, unit_of;
        std::vector<int> piece_unit_size;
        for (int32_t n = a; n < b; ++n) {
            if (sub[n] > cap) continue;
            const int32_t p = parent[n];
            if (sub[p] > cap) {
                pid[n - a] = (int32_t)roots.size();
                roots.push_back(n);
            } else {
                pid[n - a] = pid[p - a];
            }
        }
        // greedy packing in root order
        int units = 0, fill = 0;
        for (int32_t r : roots) {
            if (units == 0 || fill + sub[r] > cap) {
                ++units;
                fill = 0;
            }
            fill += sub[r];
            unit_of.push_back(units - 1);
        }
        std::vector<std::vector<int32_t>> members(units);
        for (int32_t n = a; n < b; ++n)
            if (pid[n - a] >= 0) members[unit_of[pid[n - a]]].push_back(n);
        for (int k = 0; k < units; ++k) {
            recs.clear();
            int nl = 0;
            for (int32_t n : members[k]) {
                const int32_t p = parent[n];
                const bool root = sub[p] > cap;
                pos[n] = place(n, root ? -1 : pos[p], -1);
                if (root) nl = std::max(nl, ht[n]);
                else recs.push_back({ht[n], pos[n], pos[p]});
            }
            add_unit(kUnitPiece, recs, nl);
        }
        // the trunk with the piece roots as ghost leaves; heights counted
        // within the unit (a ghost is a leaf)
        std::vector<int32_t> tn;
        for (int32_t n = a; n < b; ++n)
            if (sub[n] > cap || (parent[n] >= 0 && sub[parent[n]] > cap)) tn.push_back(n);
        for (auto it = tn.rbegin(); it != tn.rend(); ++it) th[*it] = 0;
        for (auto it = tn.rbegin(); it != tn.rend(); ++it)
            if (parent[*it] >= 0) th[parent[*it]] = std::max(th[parent[*it]], th[*it] + 1);
        recs.clear();
        for (size_t k = 0; k < tn.size(); ++k) {
            const int32_t n = tn[k], p = parent[n];
            const bool ghost = sub[n] <= cap;
            const int32_t i = place(n, p >= 0 ? pos[p] : -1, ghost ? pos[n] : -1);
            if (!ghost) pos[n] = i;   // trunk nodes: their only position
            recs.push_back({th[n], i, p >= 0 ? pos[p] : i});
        }
        add_unit(kUnitTop, recs, th[a] + 1);
    }
    h.unit_elim.push_back((int32_t)h.elim_ptr.size() - 1);
    // tallest units first so that the longest chains of barriers start first
    auto by_height = [&](std::vector<int32_t> &l) {
        std::stable_sort(l.begin(), l.end(), [&](int32_t x, int32_t y) { return levels[x] > levels[y]; });
    };
    by_height(h.list_up);
    by_height(h.list_top);
    by_height(h.list_top_g);
    by_height(h.list_down);
    return "";
}

// Device layout of a CableHost (256-byte aligned arrays), then the double
// arrays: ekn, ekp (per edge record), D, R (per position), kn (per node), DV
// (per position).
constexpr int kCableIntArrays = 16;
size_t cable_layout(const CableHost &h, int64_t N, size_t *offs) {
    const std::vector<int32_t> *arr[kCableIntArrays] = {
        &h.parent, &h.pos_node, &h.pos_par, &h.pos_src, &h.elim_n, &h.elim_p, &h.elim_ptr,
        &h.unit_pos, &h.unit_elim, &h.unit_mode, &h.list_up, &h.list_top, &h.list_top_g, &h.list_down,
        &h.pos_pnode, &h.elim_run};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + std::max<size_t>(bytes, 8) + kAlign - 1) / kAlign * kAlign;
        return o;
    };
    for (int j = 0; j < kCableIntArrays; ++j) offs[j] = take(4 * arr[j]->size());
    const size_t E = h.elim_n.size(), P = h.pos_node.size(), NN = (size_t)std::max<int64_t>(N, 1);
    offs[kCableIntArrays + 0] = take(8 * E);    // ekn
    offs[kCableIntArrays + 1] = take(8 * E);    // ekp
    offs[kCableIntArrays + 2] = take(8 * P);    // D
    offs[kCableIntArrays + 3] = take(8 * P);    // R
    offs[kCableIntArrays + 4] = take(8 * NN);   // kn
    offs[kCableIntArrays + 5] = take(8 * P);    // DV
    return off;
}

// Positions of a unit whose rows and records fit the LDS a workgroup may
// take on the current device (at most kCableLdsUnitMax, for the packed
// records).
int cable_lds_nodes() {
    int dev = 0, bytes = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int b = 0;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && b > 0)
            bytes = b;
    }
    // the level-boundary table of k_cable takes 4 KiB of static LDS; a unit's
    // packed records hold 12-bit rows
    return std::min(kCableLdsUnitMax, std::max(0, (bytes - 8192) / kCableLdsBytesPerNode));
}

struct Layout {
    size_t total = 0;
    size_t inst_end = 0;           // end of the per-instance region
    size_t off_spikes = 0, off_err = 0, off_kdev = 0, off_tiles = 0;
    size_t off_ion = 0;            // cai and ica per node, when a calcium type exists
    bool has_ion = false;
    int64_t max_tile_rows = 0;
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void compute_layout(int64_t n_nodes, std::vector<SlotHost> &slots, int prec, Layout &L) {
    const size_t ss = prec == MECH_FP32_MIXED ? 4 : 8;
    size_t off = 0;
    int64_t total_inst = 0;
    for (auto &s : slots) {
        const KindDesc &K = kKinds[s.kind];
        s.np = (s.n + kPad - 1) / kPad * kPad;
        total_inst += s.n;
        s.off_ni = off; off = align_up(off + 4 * (size_t)s.np);
        s.has_gid = K.point_process;
        if (s.has_gid) { s.off_gid = off; off = align_up(off + 4 * (size_t)s.np); }
        for (int j = 0; j < K.n_state; ++j) { s.off_st[j] = off; off = align_up(off + ss * (size_t)s.np); }
        for (int j = 0; j < K.n_param; ++j) {
            s.off_par[j] = off;
            off = align_up(off + (K.param[j].is_double ? 8 : ss) * (size_t)s.np);
        }
        s.has_ica = is_ca_kind(s.kind);
        if (s.has_ica) { s.off_ica = off; off = align_up(off + ss * (size_t)s.np); }
    }
    L.inst_end = off;
    L.off_spikes = off; off = align_up(off + 4 * (size_t)std::max<int64_t>(n_nodes, 1));
    L.off_err = off; off = align_up(off + 4);
    L.off_kdev = off; off = align_up(off + 8);
    for (auto &s : slots) {
        const size_t nch = (size_t)s.np / kPad;
        s.off_carry = off;
        off = align_up(off + 4 * nch);
        off = align_up(off + 24 * nch);
    }
    L.has_ion = false;
    for (auto &s : slots) L.has_ion |= is_ca_kind(s.kind);
    if (L.has_ion) { L.off_ion = off; off = align_up(off + 16 * (size_t)std::max<int64_t>(n_nodes, 1)); }
    L.max_tile_rows = 2 * ((total_inst + kMinTileBudget - 1) / kMinTileBudget) +
                      (n_nodes + kMinTileNodes - 1) / kMinTileNodes + 2;
    L.off_tiles = off;
    off = align_up(off + 4 * (size_t)L.max_tile_rows * (1 + slots.size()));
    L.total = off;
}

}  // namespace

struct mech_ctx {
    int64_t n_nodes = 0;
    int prec = MECH_FP64;
    bool fp32 = false;
    char *buf = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    std::vector<SlotHost> slots;
    Layout L;
    Globals gl;
    NodesDev nd{};
    CableDev cable{};
    bool nodes_bound = false, clamp_bound = false, has_syn = false, cable_bound = false;
    // fused-path launch shape and tile table
    int block = 256, tile_budget = 2048, tile_nodes = 1024, blocks_per_cu = 0, launch_flags = MECH_LAUNCH_XCD_ORDER;
    int64_t n_tiles = 0, max_tile_nodes = 0;
    std::vector<int32_t> tile_rows;   // host copy of the tile table
    int n_cu = 256;
    // time-fused path: steps per launch, and the dynamic LDS its kernels may take
    int res_steps = 64;
    size_t res_lds_allowed = 0;
    // largest tile's LDS on that path per (voltage mode, shared ion), for the
    // current tile table (cleared when the table is rebuilt)
    std::map<std::pair<int, int>, size_t> res_lds_cache;
    // graphs of 1..kGraphSteps fused steps, keyed by (vmode, dt, steps)
    std::map<std::tuple<int, uint64_t, int>, hipGraphExec_t> graphs;
    std::string err;
    int static_dev = -1;           // device whose static area holds this context (mech_alloc_static)
};

namespace {

thread_local std::string g_last_error;

int fail(mech_ctx *c, int code, const char *fmt, ...) {
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    if (c) c->err = msg;
    g_last_error = msg;
    return code;
}

#define HIPCHK(c, expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((c), MECH_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

constexpr int kGraphSteps = 64;

// A roctx range over an entry point's host work; rocprofv3 --marker-trace
// attributes the kernels it enqueues to the range.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

void clear_graphs(mech_ctx *c) {
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

GlobDev make_glob(const mech_ctx *c, double dt) {
    const Globals &G = c->gl;
    GlobDev g{};
    g.q10 = std::pow(3.0, (G.celsius - 6.3) / 10.0);
    g.ena = G.ena; g.ek = G.ek; g.eh = G.eh;
    g.cao = G.cao; g.cai0 = G.cai0;
    const double R = 8.314462618, F = 96485.33212;
    g.nernst = 1e3 * R * (G.celsius + 273.15) / (2.0 * F);
    const double kappa = 1e4 * G.ca_gamma / (2.0 * F * G.ca_depth);
    g.kt_ca = kappa * G.tau_ca;
    g.e_syn = G.e_syn; g.mg = G.mg;
    g.mg_fd = std::exp(-0.062 * G.fd_dv);
    g.mg_357 = G.mg / 3.57;
    g.fd_dv = G.fd_dv;
    g.inv_fd_dv = 1.0 / G.fd_dv;
    g.vthresh = G.vthresh;
    auto peak = [](double tr, double td) {
        const double tp = tr * td / (td - tr) * std::log(td / tr);
        return 1.0 / (std::exp(-tp / td) - std::exp(-tp / tr));
    };
    g.fa = peak(G.tau_r_ampa, G.tau_d_ampa);
    g.fn = peak(G.tau_r_nmda, G.tau_d_nmda);
    g.dt = dt;
    // cnexp factor of a linear decay over dt: exp(-y), y = dt/tau, or its
    // (1,1) Pade approximant (1 - y/2)/(1 + y/2); 1 - factor in a form with no
    // cancellation for the FP32 updates
    auto factor = [&](double tau, double *f, double *omf) {
        const double y = dt / tau;
        if (G.pade_cnexp) {
            *f = (1.0 - y / 2.0) / (1.0 + y / 2.0);
            *omf = y / (1.0 + y / 2.0);
        } else {
            *f = std::exp(-y);
            *omf = -std::expm1(-y);
        }
    };
    const double taus[4] = {G.tau_r_ampa, G.tau_d_ampa, G.tau_r_nmda, G.tau_d_nmda};
    for (int j = 0; j < 4; ++j) factor(taus[j], &g.decay[j], &g.omdecay[j]);
    factor(G.tau_ca, &g.ca_decay, &g.ca_omdecay);
    g.analytic_g = G.analytic_conductance ? 1 : 0;
    g.pade = G.pade_cnexp ? 1 : 0;
    g.kappa = kappa;
    g.pump_vmax = G.pump_vmax;
    g.pump_kp = G.pump_kp;
    g.pump_rest = G.pump_vmax * (G.cai0 / (G.cai0 + G.pump_kp));
    g.buf_total = G.buf_total;
    g.buf_kon = G.buf_kon;
    g.buf_koff = G.buf_koff;
    g.inv_tau_ca = 1.0 / G.tau_ca;
    g.newton_iters = G.newton_iters;
    g.shared_ca = G.shared_ca && c->nd.cai ? 1 : 0;
    g.seed = G.event_seed;
    // fire with probability p = rate*dt: draws below floor(p * 2^64)
    const double p = G.event_rate_hz * dt * 1e-3;
    g.threshold = !(p > 0.0) ? 0 : p >= 1.0 ? UINT64_MAX : (uint64_t)std::floor(p * 18446744073709551616.0);
    return g;
}

SlotDev slot_dev(const mech_ctx *c, int s) {
    const SlotHost &h = c->slots[s];
    const KindDesc &K = kKinds[h.kind];
    SlotDev d{};
    d.kind = h.kind;
    d.n = (int)h.n;
    d.identity = h.identity ? 1 : 0;
    d.ni = (const int *)(c->buf + h.off_ni);
    d.gid = (h.has_gid && !h.perm_identity) ? (const int *)(c->buf + h.off_gid) : nullptr;
    for (int j = 0; j < K.n_state; ++j) d.st[j] = c->buf + h.off_st[j];
    for (int j = 0; j < K.n_param; ++j) d.par[j] = c->buf + h.off_par[j];
    d.ica = h.has_ica ? (void *)(c->buf + h.off_ica) : nullptr;
    return d;
}

int build_tiles(mech_ctx *c) {
    const int ns = (int)c->slots.size();
    const int row = 1 + ns;
    std::vector<int32_t> rows;
    rows.reserve(1024);
    std::vector<int64_t> ptr(ns, 0);
    auto push = [&](int64_t node) {
        rows.push_back((int32_t)node);
        for (int s = 0; s < ns; ++s) rows.push_back((int32_t)ptr[s]);
    };
    push(0);
    int64_t cost = 0, nodes = 0, max_nodes = 0;
    int64_t nxt[kMaxSlots];
    for (int64_t n = 0; n < c->n_nodes; ++n) {
        int64_t cn = 0;
        for (int s = 0; s < ns; ++s) {
            const auto &ni = c->slots[s].ni;
            nxt[s] = ptr[s];
            while (nxt[s] < (int64_t)ni.size() && ni[nxt[s]] == n) ++nxt[s];
            cn += nxt[s] - ptr[s];
        }
        if (nodes > 0 && (cost + cn > c->tile_budget || nodes >= c->tile_nodes)) {
            push(n);
            max_nodes = std::max(max_nodes, nodes);
            cost = 0;
            nodes = 0;
        }
        for (int s = 0; s < ns; ++s) ptr[s] = nxt[s];
        cost += cn;
        ++nodes;
    }
    max_nodes = std::max(max_nodes, nodes);
    push(c->n_nodes);
    const int64_t nrows = (int64_t)rows.size() / row;
    if (nrows > c->L.max_tile_rows)
        return fail(c, MECH_ERR_NOMEM, "tile table needs %lld rows, room for %lld", (long long)nrows,
                    (long long)c->L.max_tile_rows);
    c->n_tiles = c->n_nodes > 0 ? nrows - 1 : 0;
    c->max_tile_nodes = max_nodes;
    HIPCHK(c, hipMemcpyAsync(c->buf + c->L.off_tiles, rows.data(), rows.size() * 4, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->tile_rows = std::move(rows);
    c->res_lds_cache.clear();
    clear_graphs(c);
    return MECH_OK;
}

// Reject a step with unbound inputs before anything is enqueued.
int check_ready(mech_ctx *c, int vmode) {
    if (!c->nodes_bound) return fail(c, MECH_ERR_STATE, "node vectors not bound (mech_bind_nodes)");
    if (vmode == MECH_V_CLAMP && !c->clamp_bound)
        return fail(c, MECH_ERR_STATE, "clamp waveform not bound (mech_bind_clamp)");
    if ((vmode == MECH_V_ISOLATED || vmode == MECH_V_CABLE) && !c->nd.cm)
        return fail(c, MECH_ERR_STATE, "isolated and cable modes need cm (mech_bind_nodes)");
    if (vmode == MECH_V_CABLE && (!c->cable_bound || !c->nd.area))
        return fail(c, MECH_ERR_STATE, "cable mode needs mech_bind_cable and area");
    if (vmode < MECH_V_EXTERNAL || vmode > MECH_V_CABLE) return fail(c, MECH_ERR_INVAL, "bad vmode %d", vmode);
    return MECH_OK;
}

int find_slot_var(mech_ctx *c, int slot, const char *name, bool state, size_t *off, bool *is_double) {
    if (!c || !name) return fail(c, MECH_ERR_INVAL, "null argument");
    if (slot < 0 || slot >= (int)c->slots.size()) return fail(c, MECH_ERR_INVAL, "bad type slot %d", slot);
    const SlotHost &h = c->slots[slot];
    const KindDesc &K = kKinds[h.kind];
    if (state) {
        for (int j = 0; j < K.n_state; ++j)
            if (!strcmp(K.state[j], name)) { *off = h.off_st[j]; *is_double = !c->fp32; return MECH_OK; }
        if (h.has_ica && !strcmp(name, "ica")) { *off = h.off_ica; *is_double = !c->fp32; return MECH_OK; }
    } else {
        for (int j = 0; j < K.n_param; ++j)
            if (!strcmp(K.param[j].name, name)) {
                *off = h.off_par[j];
                *is_double = K.param[j].is_double || !c->fp32;
                return MECH_OK;
            }
    }
    return fail(c, MECH_ERR_INVAL, "%s has no %s '%s'", K.name, state ? "state" : "parameter", name);
}

// Copy host doubles (caller order) into a device array (internal order).
int upload_var(mech_ctx *c, int slot, size_t off, bool is_double, const double *vals, int64_t n) {
    const SlotHost &h = c->slots[slot];
    if (n != 1 && n != h.n)
        return fail(c, MECH_ERR_INVAL, "expected 1 or %lld values, got %lld", (long long)h.n, (long long)n);
    if (h.n == 0) return MECH_OK;
    std::vector<double> tmp(h.np, 0.0);
    for (int64_t i = 0; i < h.n; ++i) {
        const int64_t u = h.perm_identity ? i : h.perm[i];
        tmp[i] = n == 1 ? vals[0] : vals[u];
    }
    if (is_double) {
        HIPCHK(c, hipMemcpyAsync(c->buf + off, tmp.data(), 8 * h.np, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> f(h.np);
        for (int64_t i = 0; i < h.np; ++i) f[i] = (float)tmp[i];
        HIPCHK(c, hipMemcpyAsync(c->buf + off, f.data(), 4 * h.np, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return MECH_OK;
}

int launch_plain_phase(mech_ctx *c, bool cur, int64_t k, const GlobDev &g, int accumulate) {
    PlainArgs a{};
    a.k = k;
    a.accumulate = accumulate;
    a.err = (int *)(c->buf + c->L.off_err);
    a.g = g;
    a.nd = c->nd;
    a.atomic_scatter = (c->launch_flags & MECH_LAUNCH_PLAIN_ATOMIC) ? 1 : 0;
    if (cur && !accumulate) HIPCHK(c, launch_fill(c->nd.rhs, c->nd.d, (int)c->n_nodes, c->stream));
    if (cur && !accumulate && g.shared_ca) HIPCHK(c, launch_fill(c->nd.ica, c->nd.ica, (int)c->n_nodes, c->stream));
    for (int s = 0; s < (int)c->slots.size(); ++s) {
        a.slot = slot_dev(c, s);
        const SlotHost &h = c->slots[s];
        a.carry_node = (int *)(c->buf + h.off_carry);
        a.carry_val = (double *)(c->buf + h.off_carry + align_up(4 * ((size_t)h.np / kPad)));
        if (cur) HIPCHK(c, launch_plain_cur(c->fp32, a, c->stream));
        else HIPCHK(c, launch_plain_state(c->fp32, a, c->stream));
    }
    // the per-node calcium pools follow the gates, from this step's currents
    if (!cur && g.shared_ca) HIPCHK(c, launch_ion_pool(c->nd, g, a.err, c->stream));
    return MECH_OK;
}

FusedArgs fused_args(mech_ctx *c, const GlobDev &g, int kofs) {
    FusedArgs a{};
    for (int s = 0; s < (int)c->slots.size(); ++s) a.slot[s] = slot_dev(c, s);
    a.n_slots = (int)c->slots.size();
    a.has_syn = c->has_syn ? 1 : 0;
    for (const auto &h : c->slots) a.has_ext |= h.kind == MECH_CABUF && h.n > 0 ? 1 : 0;
    a.tiles = (const int *)(c->buf + c->L.off_tiles);
    a.n_tiles = (int)c->n_tiles;
    a.row = 1 + (int)c->slots.size();
    a.kdev = (const long long *)(c->buf + c->L.off_kdev);
    a.kofs = kofs;
    a.xcd_order = (c->launch_flags & MECH_LAUNCH_XCD_ORDER) ? 1 : 0;
    a.nontemporal = (c->launch_flags & MECH_LAUNCH_NONTEMPORAL) ? 1 : 0;
    a.err = (int *)(c->buf + c->L.off_err);
    a.g = g;
    a.nd = c->nd;
    return a;
}

int fused_grid(const mech_ctx *c) {
    int gr = (int)c->n_tiles;
    if (c->blocks_per_cu > 0) gr = (int)std::min<int64_t>(c->n_tiles, (int64_t)c->blocks_per_cu * c->n_cu);
    return gr;
}

// One fused pass; in cable mode the pass only writes rhs/d and the tree solve
// follows it on the same stream to provide v_{k+1}.
int launch_fused_phase(mech_ctx *c, int phases, int vmode, const GlobDev &g, int kofs, hipStream_t s) {
    const int vm = vmode == MECH_V_CABLE ? MECH_V_EXTERNAL : vmode;
    const int tn = (int)std::max<int64_t>(c->max_tile_nodes, 1);
    HIPCHK(c, launch_fused(c->fp32, phases, vm, fused_args(c, g, kofs), fused_grid(c), c->block, tn, s));
    if (vmode == MECH_V_CABLE && (phases & kDoCur)) HIPCHK(c, launch_cable(c->cable, c->nd, g, s));
    return MECH_OK;
}

// A graph of n (1..kGraphSteps) fused steps: pass j reads the step index
// from the device counter plus j, and the last node advances the counter by
// n, so one graph serves every chunk of that length.
int get_graph(mech_ctx *c, int vmode, double dt, const GlobDev &g, int n, hipGraphExec_t *out) {
    uint64_t bits;
    memcpy(&bits, &dt, 8);
    auto key = std::make_tuple(vmode, bits, n);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) { *out = it->second; return MECH_OK; }
    if (!c->capture_stream)
        HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = MECH_OK;
    for (int j = 0; j < n && rc == MECH_OK; ++j)
        rc = launch_fused_phase(c, kDoState | kDoCur, vmode, g, j, c->capture_stream);
    hipError_t e1 = rc == MECH_OK ? launch_bump_k((long long *)(c->buf + c->L.off_kdev), n, c->capture_stream)
                                  : hipSuccess;
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->capture_stream, &graph);
    if (rc != MECH_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, MECH_ERR_HIP, "graph capture: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(c, MECH_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    c->graphs[key] = exec;
    *out = exec;
    return MECH_OK;
}

int step_plain(mech_ctx *c, int64_t nsteps, int64_t k0, double dt, int vmode) {
    const GlobDev g = make_glob(c, dt);
    if (vmode == MECH_V_CLAMP) HIPCHK(c, launch_vclamp(c->nd, (double)k0 * dt, c->stream));
    for (int64_t k = k0; k < k0 + nsteps; ++k) {
        int rc = launch_plain_phase(c, true, k, g, 0);
        if (rc) return rc;
        if (vmode == MECH_V_CLAMP) HIPCHK(c, launch_vclamp(c->nd, (double)(k + 1) * dt, c->stream));
        if (vmode == MECH_V_ISOLATED) HIPCHK(c, launch_visolated(c->nd, g, c->stream));
        if (vmode == MECH_V_CABLE) HIPCHK(c, launch_cable(c->cable, c->nd, g, c->stream));
        rc = launch_plain_phase(c, false, k, g, 0);
        if (rc) return rc;
    }
    return MECH_OK;
}

int step_batched(mech_ctx *c, int64_t nsteps, int64_t k0, double dt, int vmode, bool use_graph) {
    const GlobDev g = make_glob(c, dt);
    long long *kdev = (long long *)(c->buf + c->L.off_kdev);
    if (vmode == MECH_V_CLAMP) HIPCHK(c, launch_vclamp(c->nd, (double)k0 * dt, c->stream));
    HIPCHK(c, launch_set_k(kdev, k0, c->stream));
    int rc = launch_fused_phase(c, kDoCur, vmode, g, 0, c->stream);
    if (rc) return rc;
    // middle passes: state(k-1) + events(k) + cur(k) for k = k0+1 .. k0+nsteps-1,
    // replayed from graphs of kGraphSteps passes and one of the remainder
    int64_t mids = nsteps - 1;
    HIPCHK(c, launch_set_k(kdev, k0 + 1, c->stream));
    while (use_graph && mids > 0) {
        const int n = (int)std::min<int64_t>(mids, kGraphSteps);
        hipGraphExec_t exec;
        rc = get_graph(c, vmode, dt, g, n, &exec);
        if (rc) return rc;
        HIPCHK(c, hipGraphLaunch(exec, c->stream));
        mids -= n;
    }
    for (int64_t j = 0; j < mids; ++j) {
        rc = launch_fused_phase(c, kDoState | kDoCur, vmode, g, (int)j, c->stream);
        if (rc) return rc;
    }
    // closing state update at v_{k0+nsteps}
    return launch_fused_phase(c, kDoState, MECH_V_EXTERNAL, g, 0, c->stream);
}

// ------------------------------------------------------ time-fused path --
// The time-fused kernels stage each kind by its compile-time shape; check
// that shape against the kind table the buffer layout was carved from.
int res_check_shapes(mech_ctx *c) {
    for (const SlotHost &h : c->slots) {
        const KindDesc &K = kKinds[h.kind];
        const KindShape ks = kind_shape(h.kind);
        int dbl = 0;
        for (int j = 0; j < K.n_param; ++j) dbl |= K.param[j].is_double ? 1 << j : 0;
        if (ks.n_state != K.n_state || ks.n_param != K.n_param || ks.param_double != dbl ||
            ks.has_ica != (h.has_ica ? 1 : 0) || ks.has_gid != (K.point_process ? 1 : 0))
            return fail(c, MECH_ERR_STATE, "internal: staged shape of kind %s differs from the kind table", K.name);
    }
    return MECH_OK;
}

// Dynamic LDS of the largest tile of the current table.
size_t res_lds_need(mech_ctx *c, int vmode, bool ion) {
    const auto key = std::make_pair(vmode, ion ? 1 : 0);
    const auto hit = c->res_lds_cache.find(key);
    if (hit != c->res_lds_cache.end()) return hit->second;
    const int ns = (int)c->slots.size(), row = 1 + ns, ss = c->fp32 ? 4 : 8;
    size_t need = 0;
    for (int64_t t = 0; t < c->n_tiles; ++t) {
        const int32_t *r0 = c->tile_rows.data() + (size_t)t * row, *r1 = r0 + row;
        size_t b = res_node_bytes(r1[0] - r0[0], vmode, c->has_syn, ion);
        for (int s = 0; s < ns; ++s) b += res_slot_bytes(c->slots[s].kind, r1[1 + s] - r0[1 + s], ss);
        need = std::max(need, b);
    }
    c->res_lds_cache[key] = need;
    return need;
}

size_t device_lds_bytes() {
    int dev = 0, bytes = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int b = 0;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && b > 0)
            bytes = b;
    }
    return (size_t)bytes;
}

int step_resident(mech_ctx *c, int64_t nsteps, int64_t k0, double dt, int vmode) {
    if (vmode != MECH_V_CLAMP && vmode != MECH_V_ISOLATED)
        return fail(c, MECH_ERR_INVAL, "the time-fused path provides v itself: clamp or isolated mode only");
    int rc = res_check_shapes(c);
    if (rc) return rc;
    const GlobDev g = make_glob(c, dt);
    ResArgs r{};
    const size_t need = res_lds_need(c, vmode, g.shared_ca != 0), cap = device_lds_bytes();
    if (need > cap)
        return fail(c, MECH_ERR_STATE,
                    "a tile needs %zu B of LDS on the time-fused path, the device allows %zu: lower "
                    "tile_instances or tile_nodes (mech_set_launch)",
                    need, cap);
    if (need > c->res_lds_allowed) {
        HIPCHK(c, resident_allow_lds(cap));
        c->res_lds_allowed = cap;
    }
    if (vmode == MECH_V_CLAMP) HIPCHK(c, launch_vclamp(c->nd, (double)k0 * dt, c->stream));
    const FusedArgs a = fused_args(c, g, 0);
    for (int64_t done = 0; done < nsteps;) {
        const int n = (int)std::min<int64_t>(c->res_steps, nsteps - done);
        r.k0 = k0 + done;
        r.nsub = n;
        r.first_state = done > 0 ? 1 : 0;
        r.last_state = done + n == nsteps ? 1 : 0;
        HIPCHK(c, launch_resident(c->fp32, vmode, a, r, fused_grid(c), c->block, need, c->stream));
        done += n;
    }
    return MECH_OK;
}

// ------------------------------------------------- static device area --
// Device memory of the contexts made by mech_alloc_static, for callers that
// cannot allocate.  One array per device: every device the library runs on
// holds its copy until the process ends.  In host code `scratch` only names
// the symbol; its address on a device comes from hipGetSymbolAddress, taken
// once per device with that device current and kept in g_static.
constexpr int kMaxDevices = 64;

struct StaticArea {
    char *ptr = nullptr;           // device address of `scratch` on this device
    bool in_use = false;           // a live context occupies it
};
std::mutex g_static_mu;
StaticArea g_static[kMaxDevices];

void static_release(int dev) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (dev >= 0 && dev < kMaxDevices) g_static[dev].in_use = false;
}

}  // namespace

// ================================================================ C ABI ==
extern "C" {

const char *mech_strerror(int code) {
    switch (code) {
    case MECH_OK: return "ok";
    case MECH_ERR_INVAL: return "invalid argument";
    case MECH_ERR_RANGE: return "node index out of range";
    case MECH_ERR_NOMEM: return "device buffer too small";
    case MECH_ERR_STATE: return "call out of order";
    case MECH_ERR_HIP: return "HIP runtime error";
    case MECH_ERR_NONFINITE: return "non-finite state";
    default: return "unknown error";
    }
}

const char *mech_last_error(const mech_ctx *c) { return c ? c->err.c_str() : g_last_error.c_str(); }

static int validate_types(int64_t n_nodes, const mech_type_desc *types, int n_types, int prec) {
    if (n_nodes < 0 || n_nodes >= (int64_t(1) << 31)) return fail(nullptr, MECH_ERR_INVAL, "bad n_nodes");
    if (n_types < 0 || n_types > kMaxSlots) return fail(nullptr, MECH_ERR_INVAL, "n_types must be 0..%d", kMaxSlots);
    if (n_types > 0 && !types) return fail(nullptr, MECH_ERR_INVAL, "null types");
    if (prec != MECH_FP64 && prec != MECH_FP32_MIXED) return fail(nullptr, MECH_ERR_INVAL, "bad precision %d", prec);
    for (int s = 0; s < n_types; ++s) {
        if (types[s].kind < MECH_PAS || types[s].kind > MECH_CABUF)
            return fail(nullptr, MECH_ERR_INVAL, "type %d: bad kind %d", s, types[s].kind);
        if (types[s].count < 0 || types[s].count >= (int64_t(1) << 31))
            return fail(nullptr, MECH_ERR_INVAL, "type %d: bad count", s);
        if (types[s].count > 0 && !types[s].node_index)
            return fail(nullptr, MECH_ERR_INVAL, "type %d: null node_index", s);
    }
    return MECH_OK;
}

int mech_required_bytes(int64_t n_nodes, const mech_type_desc *types, int n_types, int prec, size_t *out) {
    int rc = validate_types(n_nodes, types, n_types, prec);
    if (rc) return rc;
    if (!out) return fail(nullptr, MECH_ERR_INVAL, "null out");
    std::vector<SlotHost> slots(n_types);
    for (int s = 0; s < n_types; ++s) { slots[s].kind = types[s].kind; slots[s].n = types[s].count; }
    Layout L;
    compute_layout(n_nodes, slots, prec, L);
    *out = L.total;
    return MECH_OK;
}

int mech_alloc(mech_ctx **out, int64_t n_nodes, const mech_type_desc *types, int n_types, int prec,
               void *dev_buf, size_t dev_bytes, void *hip_stream) {
    if (!out) return fail(nullptr, MECH_ERR_INVAL, "null out");
    *out = nullptr;
    int rc = validate_types(n_nodes, types, n_types, prec);
    if (rc) return rc;
    if (!dev_buf || ((uintptr_t)dev_buf % kAlign) != 0)
        return fail(nullptr, MECH_ERR_INVAL, "device buffer must be non-null and %d-byte aligned", kAlign);
    mech_ctx *c = new (std::nothrow) mech_ctx();
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "host allocation failed");
    c->n_nodes = n_nodes;
    c->prec = prec;
    c->fp32 = prec == MECH_FP32_MIXED;
    c->buf = (char *)dev_buf;
    c->bytes = dev_bytes;
    c->stream = (hipStream_t)hip_stream;
    c->slots.resize(n_types);
    for (int s = 0; s < n_types; ++s) {
        SlotHost &h = c->slots[s];
        h.kind = types[s].kind;
        h.n = types[s].count;
        if (h.kind == MECH_SYN) c->has_syn = true;
        const int32_t *ni = types[s].node_index;
        // range check, sortedness, identity
        bool sorted = true, ident = h.n == n_nodes;
        for (int64_t i = 0; i < h.n; ++i) {
            if (ni[i] < 0 || ni[i] >= n_nodes) {
                int code = fail(nullptr, MECH_ERR_RANGE, "type %d instance %lld: node %d outside [0, %lld)", s,
                                (long long)i, ni[i], (long long)n_nodes);
                delete c;
                return code;
            }
            if (i > 0 && ni[i] < ni[i - 1]) sorted = false;
            if (ni[i] != i) ident = false;
        }
        h.identity = ident;
        if (sorted) {
            h.perm_identity = true;
            h.ni.assign(ni, ni + h.n);
        } else {
            // stable counting sort by node
            h.perm_identity = false;
            std::vector<int64_t> cnt(n_nodes + 1, 0);
            for (int64_t i = 0; i < h.n; ++i) ++cnt[ni[i] + 1];
            for (int64_t n = 0; n < n_nodes; ++n) cnt[n + 1] += cnt[n];
            h.perm.resize(h.n);
            h.ni.resize(h.n);
            for (int64_t i = 0; i < h.n; ++i) {
                const int64_t p = cnt[ni[i]]++;
                h.perm[p] = (int32_t)i;
                h.ni[p] = ni[i];
            }
        }
    }
    {
        // the fused paths sum a node's contributions in fixed point, exact up
        // to kMaxPerNode of them
        std::vector<int32_t> per(n_nodes, 0);
        for (const SlotHost &h : c->slots)
            for (int32_t n : h.ni)
                if (++per[n] > kMaxPerNode) {
                    int code = fail(nullptr, MECH_ERR_INVAL, "node %d carries more than %d instances", n,
                                    kMaxPerNode);
                    delete c;
                    return code;
                }
    }
    compute_layout(n_nodes, c->slots, prec, c->L);
    if (dev_bytes < c->L.total) {
        int code = fail(nullptr, MECH_ERR_NOMEM, "device buffer has %zu bytes, %zu required", dev_bytes, c->L.total);
        delete c;
        return code;
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            c->n_cu = cu;
    }
    // upload index arrays (padded lanes point at node 0 and are never read)
    for (int s = 0; s < n_types && rc == MECH_OK; ++s) {
        SlotHost &h = c->slots[s];
        std::vector<int32_t> tmp(h.np, 0);
        std::copy(h.ni.begin(), h.ni.end(), tmp.begin());
        hipError_t e = hipMemcpy(c->buf + h.off_ni, tmp.data(), 4 * h.np, hipMemcpyHostToDevice);
        if (e == hipSuccess && h.has_gid) {
            for (int64_t i = 0; i < h.n; ++i) tmp[i] = h.perm_identity ? (int32_t)i : h.perm[i];
            e = hipMemcpy(c->buf + h.off_gid, tmp.data(), 4 * h.np, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) rc = fail(c, MECH_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
        const KindDesc &K = kKinds[h.kind];
        for (int j = 0; j < K.n_param && rc == MECH_OK; ++j) {
            size_t off;
            bool isd;
            rc = find_slot_var(c, s, K.param[j].name, false, &off, &isd);
            if (rc == MECH_OK) rc = upload_var(c, s, off, isd, &K.defaults[j], 1);
        }
    }
    if (rc == MECH_OK) {
        // the fused kernels' node accumulators take 48 B of LDS per tile node
        // (72 B under the shared calcium ion), beyond the default 64 KiB at
        // the largest tiles
        hipError_t e = fused_allow_lds(fused_lds_bytes(kMaxTileNodes, true));
        if (e != hipSuccess) rc = fail(c, MECH_ERR_HIP, "fused kernels' LDS limit: %s", hipGetErrorString(e));
    }
    if (rc == MECH_OK) {
        hipError_t e = launch_set_k((long long *)(c->buf + c->L.off_kdev), 0, c->stream);
        if (e == hipSuccess) e = launch_fill_int((int *)(c->buf + c->L.off_err), 1, c->stream);
        if (e == hipSuccess) e = launch_fill_int((int *)(c->buf + c->L.off_spikes), (int)std::max<int64_t>(n_nodes, 1), c->stream);
        if (e != hipSuccess) rc = fail(c, MECH_ERR_HIP, "init fill: %s", hipGetErrorString(e));
    }
    if (rc == MECH_OK) {
        c->nd.n_nodes = (int)n_nodes;
        c->nd.spikes = (int *)(c->buf + c->L.off_spikes);
        if (c->L.has_ion) {
            c->nd.cai = (double *)(c->buf + c->L.off_ion);
            c->nd.ica = c->nd.cai + std::max<int64_t>(n_nodes, 1);
        }
        rc = build_tiles(c);
    }
    if (rc != MECH_OK) {
        g_last_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return MECH_OK;
}

int mech_alloc_static(mech_ctx **out, int64_t n_nodes, const mech_type_desc *types, int n_types, int prec,
                      void *hip_stream) {
    if (!out) return fail(nullptr, MECH_ERR_INVAL, "null out");
    *out = nullptr;
    size_t need = 0;
    int rc = mech_required_bytes(n_nodes, types, n_types, prec, &need);
    if (rc) return rc;
    if (need > kStaticBytes)
        return fail(nullptr, MECH_ERR_NOMEM, "the context needs %zu bytes; the static area holds %zu (use mech_alloc)",
                    need, kStaticBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, MECH_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, MECH_ERR_INVAL, "device %d beyond %d", dev, kMaxDevices);
    std::unique_lock<std::mutex> lock(g_static_mu);
    StaticArea &a = g_static[dev];
    if (!a.ptr) {
        // once per device, with that device current
        char *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, MECH_ERR_HIP, "hipGetSymbolAddress: %s", hipGetErrorString(e));
        a.ptr = p;
    }
    if (a.in_use)
        return fail(nullptr, MECH_ERR_STATE, "the static area of device %d holds a live context (mech_free it first)",
                    dev);
    a.in_use = true;
    lock.unlock();
    rc = mech_alloc(out, n_nodes, types, n_types, prec, a.ptr, kStaticBytes, hip_stream);
    if (rc) {
        static_release(dev);
        return rc;
    }
    (*out)->static_dev = dev;
    return MECH_OK;
}

int mech_bind_nodes(mech_ctx *c, double *v, double *rhs, double *d, const double *area, const double *cm) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (c->n_nodes > 0 && (!v || !rhs || !d)) return fail(c, MECH_ERR_INVAL, "v, rhs and d are required");
    if (c->has_syn && c->n_nodes > 0 && !area) return fail(c, MECH_ERR_INVAL, "area is required with synapses");
    c->nd.v = v;
    c->nd.rhs = rhs;
    c->nd.d = d;
    c->nd.area = area;
    c->nd.cm = cm;
    c->nodes_bound = true;
    clear_graphs(c);
    return MECH_OK;
}

// The unit size bound for a requested unit_nodes, at most the device's LDS
// capacity; the fallback capacity is the one without the large-LDS opt-in.
// The default, 1024 nodes, was the fastest bound on branched cells of 200 to
// 20 000 compartments (units of 512 to 4096 nodes measured): smaller units
// run more workgroups at once, larger ones leave fewer trunk heights.
constexpr int kCableFallbackNodes = (65536 - 8192) / kCableLdsBytesPerNode;
constexpr int kCableDefaultUnit = 1024;
int cable_cap(int32_t unit_nodes, int lds_nodes) {
    return std::min<int>(unit_nodes > 0 ? unit_nodes : kCableDefaultUnit, lds_nodes);
}

int mech_cable_required_bytes(int64_t n_nodes, const int32_t *parent, int32_t unit_nodes, size_t *out) {
    if (!out || n_nodes < 0 || (n_nodes > 0 && !parent) || unit_nodes < 0)
        return fail(nullptr, MECH_ERR_INVAL, "null argument or negative unit_nodes");
    size_t need = 0, offs[kCableIntArrays + 6];
    // mech_bind_cable cuts with the device's capacity, or with the fallback
    // if the device refuses the large LDS request: size for both
    for (int lds : {std::max(cable_lds_nodes(), 1), kCableFallbackNodes}) {
        CableHost h;
        std::string why = build_cable(n_nodes, parent, cable_cap(unit_nodes, lds), h);
        if (!why.empty()) return fail(nullptr, MECH_ERR_INVAL, "%s", why.c_str());
        need = std::max(need, cable_layout(h, n_nodes, offs));
    }
    *out = need;
    return MECH_OK;
}

int mech_cable_plan(int64_t n_nodes, const int32_t *parent, int32_t unit_nodes, int32_t *sizes, int32_t *buf,
                    int64_t buf_len) {
    if (!sizes || n_nodes < 0 || (n_nodes > 0 && !parent) || unit_nodes < 0 || buf_len < 0)
        return fail(nullptr, MECH_ERR_INVAL, "null argument or negative size");
    CableHost h;
    std::string why = build_cable(n_nodes, parent, cable_cap(unit_nodes, std::max(cable_lds_nodes(), 1)), h);
    if (!why.empty()) return fail(nullptr, MECH_ERR_INVAL, "%s", why.c_str());
    constexpr int kPlanArrays = 14;   // pos_pnode (parent of pos_node) is not part of the plan
    const std::vector<int32_t> *arr[kPlanArrays] = {
        &h.parent, &h.pos_node, &h.pos_par, &h.pos_src, &h.elim_n, &h.elim_p, &h.elim_ptr,
        &h.unit_pos, &h.unit_elim, &h.unit_mode, &h.list_up, &h.list_top, &h.list_top_g, &h.list_down};
    int64_t total = 0;
    for (int j = 0; j < kPlanArrays; ++j) {
        sizes[j] = (int32_t)arr[j]->size();
        total += sizes[j];
    }
    if (!buf) return MECH_OK;
    if (buf_len < total) return fail(nullptr, MECH_ERR_NOMEM, "plan needs %lld entries", (long long)total);
    for (int j = 0; j < kPlanArrays; ++j) buf = std::copy(arr[j]->begin(), arr[j]->end(), buf);
    return MECH_OK;
}

int mech_bind_cable(mech_ctx *c, const int32_t *parent, const double *g_axial, int32_t unit_nodes, void *dev_buf,
                    size_t dev_bytes) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (c->n_nodes > 0 && (!parent || !g_axial || !dev_buf))
        return fail(c, MECH_ERR_INVAL, "parent, g_axial and dev_buf are required");
    if (unit_nodes < 0) return fail(c, MECH_ERR_INVAL, "unit_nodes must be >= 0");
    if (((uintptr_t)dev_buf % kAlign) != 0) return fail(c, MECH_ERR_INVAL, "dev_buf must be %d-byte aligned", kAlign);
    int lds_nodes = std::max(cable_lds_nodes(), 1);
    if (lds_nodes * kCableLdsBytesPerNode > 65536 &&
        cable_allow_lds((size_t)lds_nodes * kCableLdsBytesPerNode) != hipSuccess) {
        (void)hipGetLastError();
        lds_nodes = kCableFallbackNodes;
    }
    CableHost h;
    std::string why = build_cable(c->n_nodes, parent, cable_cap(unit_nodes, lds_nodes), h);
    if (!why.empty()) return fail(c, MECH_ERR_INVAL, "%s", why.c_str());
    size_t offs[kCableIntArrays + 6];
    const size_t need = cable_layout(h, c->n_nodes, offs);
    if (dev_bytes < need) return fail(c, MECH_ERR_NOMEM, "cable buffer has %zu bytes, %zu required", dev_bytes, need);
    char *b = (char *)dev_buf;
    const std::vector<int32_t> *arr[kCableIntArrays] = {
        &h.parent, &h.pos_node, &h.pos_par, &h.pos_src, &h.elim_n, &h.elim_p, &h.elim_ptr,
        &h.unit_pos, &h.unit_elim, &h.unit_mode, &h.list_up, &h.list_top, &h.list_top_g, &h.list_down,
        &h.pos_pnode, &h.elim_run};
    for (int j = 0; j < kCableIntArrays; ++j)
        if (!arr[j]->empty())
            HIPCHK(c, hipMemcpy(b + offs[j], arr[j]->data(), 4 * arr[j]->size(), hipMemcpyHostToDevice));
    const int *I[kCableIntArrays];
    for (int j = 0; j < kCableIntArrays; ++j) I[j] = (const int *)(b + offs[j]);
    CableDev d{};
    d.g_axial = g_axial;
    d.parent = I[0];
    d.pos_node = I[1];
    d.pos_par = I[2];
    d.pos_src = I[3];
    d.elim_n = I[4];
    d.elim_p = I[5];
    d.elim_ptr = I[6];
    d.unit_pos = I[7];
    d.unit_elim = I[8];
    d.unit_mode = I[9];
    d.list_up = I[10];
    d.list_top = I[11];
    d.list_top_g = I[12];
    d.list_down = I[13];
    d.pos_pnode = I[14];
    d.elim_run = I[15];
    d.n_up = (int)h.list_up.size();
    d.n_top = (int)h.list_top.size();
    d.n_top_g = (int)h.list_top_g.size();
    d.n_down = (int)h.list_down.size();
    d.lds_max_nodes = h.lds_max;
    d.ekn = (double *)(b + offs[kCableIntArrays + 0]);
    d.ekp = (double *)(b + offs[kCableIntArrays + 1]);
    d.D = (double *)(b + offs[kCableIntArrays + 2]);
    d.R = (double *)(b + offs[kCableIntArrays + 3]);
    d.kn = (double *)(b + offs[kCableIntArrays + 4]);
    d.DV = (double *)(b + offs[kCableIntArrays + 5]);
    if (c->n_nodes > 0) {
        if (!c->nd.area) return fail(c, MECH_ERR_STATE, "bind area (mech_bind_nodes) before mech_bind_cable");
        HIPCHK(c, launch_cable_coeffs(d, c->nd.area, (int)c->n_nodes, (int)h.elim_n.size(), c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->cable = d;
    c->cable_bound = true;
    clear_graphs(c);
    return MECH_OK;
}

int mech_bind_clamp(mech_ctx *c, const double *off, const double *amp, const double *freq, const double *phase) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (c->n_nodes > 0 && (!off || !amp || !freq || !phase))
        return fail(c, MECH_ERR_INVAL, "all four clamp arrays are required");
    c->nd.c_off = off;
    c->nd.c_amp = amp;
    c->nd.c_freq = freq;
    c->nd.c_phase = phase;
    c->clamp_bound = true;
    clear_graphs(c);
    return MECH_OK;
}

int mech_set_params(mech_ctx *c, int slot, const char *name, const double *vals, int64_t n) {
    if (!c || !vals) return fail(c, MECH_ERR_INVAL, "null argument");
    size_t off;
    bool isd;
    int rc = find_slot_var(c, slot, name, false, &off, &isd);
    if (rc) return rc;
    return upload_var(c, slot, off, isd, vals, n);
}

int mech_set_global(mech_ctx *c, const char *name, double value) {
    if (!c || !name) return fail(c, MECH_ERR_INVAL, "null argument");
    Globals &G = c->gl;
    struct { const char *n; double *p; } tab[] = {
        {"celsius", &G.celsius}, {"ena", &G.ena}, {"ek", &G.ek}, {"eh", &G.eh}, {"cao", &G.cao},
        {"cai0", &G.cai0}, {"tau_ca", &G.tau_ca}, {"ca_gamma", &G.ca_gamma}, {"ca_depth", &G.ca_depth},
        {"e_syn", &G.e_syn}, {"mg", &G.mg}, {"tau_r_ampa", &G.tau_r_ampa}, {"tau_d_ampa", &G.tau_d_ampa},
        {"tau_r_nmda", &G.tau_r_nmda}, {"tau_d_nmda", &G.tau_d_nmda}, {"event_rate_hz", &G.event_rate_hz},
        {"vthresh", &G.vthresh}, {"fd_dv", &G.fd_dv}, {"pump_vmax", &G.pump_vmax}, {"pump_kp", &G.pump_kp},
        {"buf_total", &G.buf_total}, {"buf_kon", &G.buf_kon}, {"buf_koff", &G.buf_koff}};
    if (!strcmp(name, "newton_iters")) {
        if (!(value >= 1.0 && value <= 16.0) || value != std::floor(value))
            return fail(c, MECH_ERR_INVAL, "newton_iters must be an integer in [1, 16]");
        G.newton_iters = (int)value;
        clear_graphs(c);
        return MECH_OK;
    }
    if (!strcmp(name, "event_seed")) {
        if (!(value >= 0.0) || value >= 9007199254740992.0 || value != std::floor(value))
            return fail(c, MECH_ERR_INVAL, "event_seed must be an integer in [0, 2^53)");
        G.event_seed = (uint64_t)value;
        clear_graphs(c);
        return MECH_OK;
    }
    if (!strcmp(name, "shared_ca")) {
        if (value != 0.0 && value != 1.0) return fail(c, MECH_ERR_INVAL, "shared_ca must be 0 or 1");
        if (value != 0.0 && !c->nd.cai)
            return fail(c, MECH_ERR_STATE, "shared_ca needs a cahva, capump or cabuf type");
        G.shared_ca = value != 0.0;
        clear_graphs(c);
        return MECH_OK;
    }
    if (!strcmp(name, "analytic_conductance") || !strcmp(name, "pade_cnexp")) {
        if (value != 0.0 && value != 1.0) return fail(c, MECH_ERR_INVAL, "%s must be 0 or 1", name);
        (name[0] == 'a' ? G.analytic_conductance : G.pade_cnexp) = value != 0.0;
        clear_graphs(c);
        return MECH_OK;
    }
    for (auto &t : tab)
        if (!strcmp(t.n, name)) {
            if (!std::isfinite(value)) return fail(c, MECH_ERR_INVAL, "%s must be finite", name);
            *t.p = value;
            clear_graphs(c);
            return MECH_OK;
        }
    return fail(c, MECH_ERR_INVAL, "unknown global '%s'", name);
}

int mech_init(mech_ctx *c) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (!c->nodes_bound) return fail(c, MECH_ERR_STATE, "node vectors not bound (mech_bind_nodes)");
    TraceRange range("mech_init");
    PlainArgs a{};
    a.err = (int *)(c->buf + c->L.off_err);
    a.g = make_glob(c, 0.025);
    a.nd = c->nd;
    for (int s = 0; s < (int)c->slots.size(); ++s) {
        a.slot = slot_dev(c, s);
        HIPCHK(c, launch_init(c->fp32, a, c->stream));
    }
    HIPCHK(c, launch_fill_int(c->nd.spikes, (int)std::max<int64_t>(c->n_nodes, 1), c->stream));
    if (c->nd.cai) HIPCHK(c, launch_ion_init(c->nd, a.g, c->stream));
    return MECH_OK;
}

int mech_cur(mech_ctx *c, int64_t k, double dt, int accumulate) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    int rc = check_ready(c, MECH_V_EXTERNAL);
    if (rc) return rc;
    if (!(dt > 0.0) || k < 0) return fail(c, MECH_ERR_INVAL, "need dt > 0 and k >= 0");
    TraceRange range("mech_cur");
    return launch_plain_phase(c, true, k, make_glob(c, dt), accumulate);
}

int mech_state(mech_ctx *c, double dt) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    int rc = check_ready(c, MECH_V_EXTERNAL);
    if (rc) return rc;
    if (!(dt > 0.0)) return fail(c, MECH_ERR_INVAL, "need dt > 0");
    TraceRange range("mech_state");
    return launch_plain_phase(c, false, 0, make_glob(c, dt), 0);
}

int mech_step(mech_ctx *c, int64_t nsteps, int64_t k0, double dt, int vmode, int path) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    int rc = check_ready(c, vmode);
    if (rc) return rc;
    if (!(dt > 0.0) || k0 < 0 || nsteps < 0 || k0 + nsteps >= (int64_t(1) << 32))
        return fail(c, MECH_ERR_INVAL, "need dt > 0, k0 >= 0, nsteps >= 0, k0 + nsteps < 2^32");
    if (nsteps == 0) return MECH_OK;
    static const char *const kRange[] = {"mech_step plain", "mech_step batched", "mech_step resident"};
    TraceRange range(path >= 0 && path <= MECH_PATH_RESIDENT ? kRange[path] : "mech_step");
    if (path == MECH_PATH_PLAIN) return step_plain(c, nsteps, k0, dt, vmode);
    if (path == MECH_PATH_BATCHED) return step_batched(c, nsteps, k0, dt, vmode, true);
    if (path == MECH_PATH_RESIDENT) return step_resident(c, nsteps, k0, dt, vmode);
    return fail(c, MECH_ERR_INVAL, "bad path %d", path);
}

int mech_set_resident_steps(mech_ctx *c, int steps_per_launch) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (steps_per_launch < 1 || steps_per_launch > 4096)
        return fail(c, MECH_ERR_INVAL, "steps_per_launch must be in [1, 4096]");
    c->res_steps = steps_per_launch;
    return MECH_OK;
}

int mech_set_launch(mech_ctx *c, int block, int tile_instances, int tile_nodes, int blocks_per_cu, int flags) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (flags & ~(MECH_LAUNCH_XCD_ORDER | MECH_LAUNCH_NONTEMPORAL | MECH_LAUNCH_PLAIN_ATOMIC))
        return fail(c, MECH_ERR_INVAL, "unknown launch flags 0x%x", flags);
    if (block < 64 || block > 1024 || block % 64)
        return fail(c, MECH_ERR_INVAL, "block must be a multiple of 64 in [64, 1024]");
    if (tile_instances < std::max(block, kMinTileBudget))
        return fail(c, MECH_ERR_INVAL, "tile_instances must be >= block");
    if (tile_nodes < kMinTileNodes || tile_nodes > kMaxTileNodes)
        return fail(c, MECH_ERR_INVAL, "tile_nodes must be in [%d, %d]", kMinTileNodes, kMaxTileNodes);
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(c, MECH_ERR_INVAL, "blocks_per_cu must be 0..64");
    c->block = block;
    c->tile_budget = tile_instances;
    c->tile_nodes = tile_nodes;
    c->blocks_per_cu = blocks_per_cu;
    c->launch_flags = flags;
    return build_tiles(c);
}

int mech_get_launch(const mech_ctx *c, int *block, int *tile_instances, int *tile_nodes, int *blocks_per_cu,
                    int *flags) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (flags) *flags = c->launch_flags;
    if (block) *block = c->block;
    if (tile_instances) *tile_instances = c->tile_budget;
    if (tile_nodes) *tile_nodes = c->tile_nodes;
    if (blocks_per_cu) *blocks_per_cu = c->blocks_per_cu;
    return MECH_OK;
}

int mech_info(const mech_ctx *c, int64_t *n_tiles, int64_t *max_tile_nodes) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    if (n_tiles) *n_tiles = c->n_tiles;
    if (max_tile_nodes) *max_tile_nodes = c->max_tile_nodes;
    return MECH_OK;
}

// Time candidate launch shapes of the batched (or time-fused) path and keep
// the fastest; everything a step writes is saved before and restored after.
static int autotune_impl(mech_ctx *c, double dt, int vmode, int nsteps, int reps, double *best_ms, bool resident) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    TraceRange range(resident ? "mech_autotune_resident" : "mech_autotune");
    int rc = check_ready(c, vmode);
    if (rc) return rc;
    if (!(dt > 0.0) || nsteps < 1 || reps < 1) return fail(c, MECH_ERR_INVAL, "need dt > 0, nsteps >= 1, reps >= 1");
    if (resident && vmode != MECH_V_CLAMP && vmode != MECH_V_ISOLATED)
        return fail(c, MECH_ERR_INVAL, "the time-fused path provides v itself: clamp or isolated mode only");
    // save everything a step writes
    const size_t nb = 8 * (size_t)c->n_nodes, ion = c->nd.cai ? 2 * nb : 0;
    const size_t save_bytes = c->L.inst_end + 3 * nb + 4 * (size_t)c->n_nodes + ion;
    char *save = nullptr;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMalloc(&save, std::max<size_t>(save_bytes, 1)));
    auto copy_all = [&](bool to_save) -> hipError_t {
        struct { void *dev; size_t n; } parts[] = {
            {c->buf, c->L.inst_end}, {c->nd.v, nb}, {c->nd.rhs, nb}, {c->nd.d, nb},
            {c->nd.spikes, 4 * (size_t)c->n_nodes}, {c->nd.cai, ion / 2}, {c->nd.ica, ion / 2}};
        size_t o = 0;
        for (auto &p : parts) {
            if (p.n == 0) continue;
            hipError_t e = to_save ? hipMemcpyAsync(save + o, p.dev, p.n, hipMemcpyDeviceToDevice, c->stream)
                                   : hipMemcpyAsync(p.dev, save + o, p.n, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return e;
            o += p.n;
        }
        return hipStreamSynchronize(c->stream);
    };
    hipError_t e = copy_all(true);
    if (e != hipSuccess) { (void)hipFree(save); return fail(c, MECH_ERR_HIP, "autotune save: %s", hipGetErrorString(e)); }
    int best[5] = {c->block, c->tile_budget, c->tile_nodes, c->blocks_per_cu, c->launch_flags};
    double best_t = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    struct Shape { int block, budget, nodes, bpc, flags; };
    std::vector<Shape> cand;
    if (!resident) {
        // the non-temporal flag measured slower on every shape tried; it
        // stays available through mech_set_launch but is not searched
        for (int b : {128, 256, 512})
            for (int ipt : {1, 2, 4, 8})
                for (int bpc : {0, 1, 2, 8})
                    for (int fl : {0, (int)MECH_LAUNCH_XCD_ORDER}) {
                        const int budget = b * ipt;
                        cand.push_back({b, budget, std::min(kMaxTileNodes, std::max(kMinTileNodes, budget)), bpc, fl});
                    }
    } else {
        // a tile stays on one CU for many steps, so its LDS (and how many
        // tiles share a CU) matters more than the stream order
        for (int b : {64, 128, 256, 512})
            for (int ipt : {1, 2, 4})
                for (int half : {0, 1}) {
                    const int budget = std::max(b * ipt, kMinTileBudget);
                    const int nodes = std::min(kMaxTileNodes, std::max(kMinTileNodes, half ? budget / 2 : budget));
                    cand.push_back({b, budget, nodes, 0, (int)MECH_LAUNCH_XCD_ORDER});
                }
    }
    const int ion_on = c->gl.shared_ca && c->nd.cai;
    const size_t cap = device_lds_bytes();
    // median ms per step of one shape over `r` runs of `n` steps; +inf if its
    // tiles do not fit the LDS of a workgroup
    auto time_shape = [&](const Shape &sh, int n, int r, double &t) -> int {
        t = 1e300;
        int q = mech_set_launch(c, sh.block, sh.budget, sh.nodes, sh.bpc, sh.flags);
        if (q) return q;
        if (resident && res_lds_need(c, vmode, ion_on) > cap) return MECH_OK;
        auto run = [&](int m, int64_t k0) {
            return resident ? step_resident(c, m, k0, dt, vmode) : step_batched(c, m, k0, dt, vmode, false);
        };
        q = run(1, 0);  // warm-up
        std::vector<double> ts;
        for (int j = 0; j < r && q == MECH_OK; ++j) {
            (void)hipEventRecord(e0, c->stream);
            q = run(n, 1);
            (void)hipEventRecord(e1, c->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ts.push_back(ms / n);
        }
        if (q) return q;
        std::sort(ts.begin(), ts.end());
        t = ts[ts.size() / 2];
        return MECH_OK;
    };
    // a first pass over every candidate, then the four fastest again with
    // four times the steps and twice the repeats (short runs rank shapes
    // within a few per cent of each other in noise)
    std::vector<std::pair<double, Shape>> timed;
    for (const Shape &sh : cand) {
        double t;
        rc = time_shape(sh, nsteps, reps, t);
        if (rc) break;
        if (t < 1e299) timed.push_back({t, sh});
    }
    if (rc == MECH_OK) {
        std::sort(timed.begin(), timed.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
        if (timed.size() > 4) timed.resize(4);
        for (auto &ts : timed) {
            if (timed.size() > 1) {
                rc = time_shape(ts.second, 4 * nsteps, 2 * reps, ts.first);
                if (rc) break;
            }
            if (ts.first < best_t) {
                best_t = ts.first;
                const Shape &sh = ts.second;
                best[0] = sh.block; best[1] = sh.budget; best[2] = sh.nodes; best[3] = sh.bpc; best[4] = sh.flags;
            }
        }
    }
    // finer tile sizes around the fastest shape (10/16 to 20/16 of its
    // budget and node span, multiples of 64): the LDS a tile takes sets how
    // many workgroups share a CU, and the coarse grid's powers of two can
    // miss the size where one more fits
    if (rc == MECH_OK && best_t < 1e299) {
        const Shape b0{best[0], best[1], best[2], best[3], best[4]};
        for (int num : {10, 11, 12, 13, 14, 15, 17, 18, 20}) {
            Shape sh = b0;
            sh.budget = std::max(std::max(b0.block, kMinTileBudget), (b0.budget * num / 16 + 63) / 64 * 64);
            sh.nodes = std::min(kMaxTileNodes, std::max(kMinTileNodes, (b0.nodes * num / 16 + 63) / 64 * 64));
            double t;
            rc = time_shape(sh, 4 * nsteps, 2 * reps, t);
            if (rc) break;
            if (t < best_t) {
                best_t = t;
                best[1] = sh.budget;
                best[2] = sh.nodes;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int rc2 = mech_set_launch(c, best[0], best[1], best[2], best[3], best[4]);
    e = copy_all(false);
    (void)hipFree(save);
    if (rc) return rc;
    if (rc2) return rc2;
    if (e != hipSuccess) return fail(c, MECH_ERR_HIP, "autotune restore: %s", hipGetErrorString(e));
    if (best_t > 1e299) return fail(c, MECH_ERR_STATE, "no candidate launch shape fits the LDS of a workgroup");
    if (best_ms) *best_ms = best_t;
    return MECH_OK;
}

int mech_autotune(mech_ctx *c, double dt, int vmode, int nsteps, int reps, double *best_ms) {
    return autotune_impl(c, dt, vmode, nsteps, reps, best_ms, false);
}

int mech_autotune_resident(mech_ctx *c, double dt, int vmode, int nsteps, int reps, double *best_ms) {
    return autotune_impl(c, dt, vmode, nsteps, reps, best_ms, true);
}

// slot -1: the per-node calcium ion ("cai", "ica"), n_nodes doubles.
static int ion_array(mech_ctx *c, const char *name, int64_t n, double **out) {
    if (!c->nd.cai) return fail(c, MECH_ERR_INVAL, "no per-node ion: the context has no calcium type");
    if (!strcmp(name, "cai")) *out = c->nd.cai;
    else if (!strcmp(name, "ica")) *out = c->nd.ica;
    else return fail(c, MECH_ERR_INVAL, "per-node ion arrays are 'cai' and 'ica', not '%s'", name);
    if (n != c->n_nodes) return fail(c, MECH_ERR_INVAL, "expected %lld nodes", (long long)c->n_nodes);
    return MECH_OK;
}

int mech_get_state(mech_ctx *c, int slot, const char *name, double *host_out, int64_t n) {
    if (!c || !host_out || !name) return fail(c, MECH_ERR_INVAL, "null argument");
    if (slot == -1) {
        double *p;
        int rc = ion_array(c, name, n, &p);
        if (rc || n == 0) return rc;
        HIPCHK(c, hipMemcpyAsync(host_out, p, 8 * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return MECH_OK;
    }
    size_t off;
    bool isd;
    int rc = find_slot_var(c, slot, name, true, &off, &isd);
    if (rc) return rc;
    const SlotHost &h = c->slots[slot];
    if (n != h.n) return fail(c, MECH_ERR_INVAL, "expected %lld values", (long long)h.n);
    if (h.n == 0) return MECH_OK;
    std::vector<double> tmp(h.n);
    if (isd) {
        HIPCHK(c, hipMemcpyAsync(tmp.data(), c->buf + off, 8 * h.n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> f(h.n);
        HIPCHK(c, hipMemcpyAsync(f.data(), c->buf + off, 4 * h.n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < h.n; ++i) tmp[i] = f[i];
    }
    for (int64_t i = 0; i < h.n; ++i) host_out[h.perm_identity ? i : h.perm[i]] = tmp[i];
    return MECH_OK;
}

int mech_set_state(mech_ctx *c, int slot, const char *name, const double *host_in, int64_t n) {
    if (!c || !host_in || !name) return fail(c, MECH_ERR_INVAL, "null argument");
    if (slot == -1) {
        double *p;
        int rc = ion_array(c, name, n, &p);
        if (rc || n == 0) return rc;
        HIPCHK(c, hipMemcpyAsync(p, host_in, 8 * n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return MECH_OK;
    }
    size_t off;
    bool isd;
    int rc = find_slot_var(c, slot, name, true, &off, &isd);
    if (rc) return rc;
    if (n != c->slots[slot].n) return fail(c, MECH_ERR_INVAL, "expected %lld values", (long long)c->slots[slot].n);
    return upload_var(c, slot, off, isd, host_in, n);
}

int mech_spike_counts(mech_ctx *c, int32_t *host_out, int64_t n) {
    if (!c || !host_out) return fail(c, MECH_ERR_INVAL, "null argument");
    if (n != c->n_nodes) return fail(c, MECH_ERR_INVAL, "expected %lld nodes", (long long)c->n_nodes);
    if (n == 0) return MECH_OK;
    HIPCHK(c, hipMemcpyAsync(host_out, c->nd.spikes, 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MECH_OK;
}

int mech_sync(mech_ctx *c) {
    if (!c) return fail(nullptr, MECH_ERR_INVAL, "null ctx");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    int flag = 0;
    HIPCHK(c, hipMemcpy(&flag, c->buf + c->L.off_err, 4, hipMemcpyDeviceToHost));
    if (flag) {
        HIPCHK(c, launch_fill_int((int *)(c->buf + c->L.off_err), 1, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return fail(c, MECH_ERR_NONFINITE, "a kernel stored a non-finite state");
    }
    return MECH_OK;
}

int mech_probe_stream(int op, int unroll, int blocks_per_cu, int flags, void *dst, const void *src, size_t bytes,
                      void *hip_stream) {
    if (op < 0 || op > 6 || (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) || blocks_per_cu < 1 ||
        blocks_per_cu > 64 || flags < 0 || flags > 63)
        return fail(nullptr, MECH_ERR_INVAL, "probe: op 0..6, unroll 1/2/4/8, blocks_per_cu 1..64, flags 0..63");
    if (!dst || (op != 2 && op < 5 && !src) || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(nullptr, MECH_ERR_INVAL, "probe needs 16-byte aligned buffers and size");
    if (op == 5 && (bytes % 56 || (bytes / 56) % 256))
        return fail(nullptr, MECH_ERR_INVAL, "probe op 5: bytes must be 56 times a multiple of 256");
    if (op == 6 && (bytes % 160 || (bytes / 160) % 2048))
        return fail(nullptr, MECH_ERR_INVAL, "probe op 6: bytes must be 160 times a multiple of 2048");
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    int grid = blocks_per_cu * cu;
    if (op == 4) grid += grid & 1;   // a reading and a writing half
    hipError_t e = launch_stream(op, unroll, flags, dst, src, bytes, grid, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, MECH_ERR_HIP, "probe: %s", hipGetErrorString(e));
    return MECH_OK;
}

void mech_free(mech_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    clear_graphs(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->static_dev >= 0) static_release(c->static_dev);
    delete c;
}

}  // extern "C"
