// mech_internal.h -- structures shared by the host runtime and the kernels of
// libmech.so.  Not part of the public interface (include/mech.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mech.h"

namespace mech {

constexpr int kMaxSlots = 8;
constexpr int kMaxStates = 4;
constexpr int kMaxParams = 4;
constexpr int kPad = 64;             // instances per padding unit (one wave)
constexpr int kAlign = 256;          // byte alignment of every carved array
constexpr int kMinTileBudget = 64;   // smallest tile work budget (instances)
constexpr int kMinTileNodes = 64;
constexpr int kMaxPerNode = 1 << 19; // instances on one node: the fused paths' fixed-point node sums stay exact
constexpr int kMaxTileNodes = 2048;  // LDS: 48 B per node -> 96 KiB per block (144 KiB with the shared calcium ion)

// Step-phase flags of the fused kernel.
enum : int { kDoState = 1, kDoCur = 2 };
// Kinds that carry a calcium current and a pool (Ca-HVA gates).
constexpr bool is_ca_kind(int kind) { return kind == MECH_CAHVA || kind == MECH_CAPUMP || kind == MECH_CABUF; }

// One mechanism type as the kernels see it (internal, node-sorted order).
// Storage types: S = state type (double or float); conductance PARAMETERs
// are S as well; reversal potentials, weights and node data are double.
struct SlotDev {
    int kind;
    int n;                     // instances
    int identity;              // node_index[i] == i for all i and n == n_nodes
    const int *ni;             // node index per instance
    const int *gid;            // synapse event-stream id (nullptr: instance index)
    void *st[kMaxStates];      // STATE arrays
    const void *par[kMaxParams];
    void *ica;                 // Ca-HVA current (S)
};

// Globals with every dt-dependent constant precomputed on the host in FP64.
struct GlobDev {
    double q10;                // hh temperature factor 3^((celsius-6.3)/10)
    double ena, ek, eh;
    double cao, cai0;
    double nernst;             // 1e3 R T / (2 F), mV
    double kt_ca;              // kappa * tau_ca
    double e_syn, mg;
    double mg_fd;              // exp(-0.062 fd_dv)
    double mg_357;             // mg / 3.57
    double fd_dv, inv_fd_dv, vthresh;
    double fa, fn;             // synapse peak-normalisation factors
    double dt;
    double decay[4];           // exp(-dt/tau) of A_ampa, B_ampa, A_nmda, B_nmda
    double omdecay[4];         // 1 - decay, from expm1
    double ca_decay, ca_omdecay;
    uint64_t seed, threshold;  // event draws: fire when H(seed, gid, k) < threshold
    int analytic_g;            // conductance in closed form instead of the finite difference
    int pade;                  // cnexp factor exp(-y) replaced by (1 - y/2)/(1 + y/2)
    double kappa;              // calcium influx per unit current, mM/ms per mA/cm2
    double pump_vmax, pump_kp, pump_rest;   // pump_rest = vmax cai0/(cai0 + kp)
    int newton_iters;
    int shared_ca;             // calcium as a per-node ion (NodesDev::cai, ica)
    double buf_total, buf_kon, buf_koff;   // cabuf's buffer (mM, 1/(mM ms), 1/ms)
    double inv_tau_ca;                     // 1/tau_ca
};

struct NodesDev {
    double *v, *rhs, *d;
    const double *area, *cm;
    const double *c_off, *c_amp, *c_freq, *c_phase;
    int *spikes;
    int n_nodes;
    // per-node calcium ion (library region; null without a calcium type):
    // concentration (mM) and the total calcium current density (mA/cm2) of
    // the last current update, used when GlobDev::shared_ca is set
    double *cai, *ica;
};

// Cell trees of the cable mode, cut into units that one workgroup solves.
// A unit is a whole cell (FULL), a forest of subtrees whose roots hang off a
// larger cell's trunk (PIECE), or that trunk (TOP) with the piece roots as
// ghost rows.  Rows of the solve live at positions: every node has one, and
// every piece root has a second one as a ghost in its trunk's unit.
enum { kUnitFull = 0, kUnitPiece = 1, kUnitTop = 2 };
// LDS of a unit solved there, per position: D, R and the voltage difference
// to the parent (24 B) and one edge record (packed rows and run length, two
// couplings: 20 B).
constexpr int kCableLdsBytesPerNode = 44;
// A unit solved in LDS packs each record as child row (12 bits), parent row
// (12 bits) and run length (8 bits): at most 4095 rows, runs of up to
// kCableRunMax children of one parent at one height per head (a longer run
// is followed by comparing parents).
constexpr int kCableLdsUnitMax = 4095;
constexpr int kCableRunMax = 255;

struct CableDev {
    const double *g_axial;     // uS to the parent
    const int *parent;         // [n_nodes]
    const int *pos_node;       // [n_pos] node of each position
    const int *pos_pnode;      // [n_pos] that node's parent node, or -1
    const int *pos_par;        // [n_pos] position of the parent's row in the same unit, or -1
    const int *pos_src;        // [n_pos] ghost: the piece root's own position; -1 otherwise
    const int *elim_run;       // per record: run length at the head of a parent's run of a height, else 0
    const int *elim_n;         // edge records: child position, per unit by the child's height
    const int *elim_p;         // parent position
    const int *elim_ptr;       // height boundaries into elim_n / elim_p
    const int *unit_pos;       // [n_units + 1] position ranges
    const int *unit_elim;      // [n_units + 1] into elim_ptr
    const int *unit_mode;      // [n_units] kUnit*
    const int *list_up;        // FULL and PIECE units (LDS), tallest first
    const int *list_top;       // TOP units that fit in LDS
    const int *list_top_g;     // TOP units solved in global scratch
    const int *list_down;      // FULL and PIECE units, second pass (back-substitution)
    int n_up, n_top, n_top_g, n_down;
    int lds_max_nodes;         // largest unit solved in LDS
    double *ekn, *ekp;         // per edge record: 100 g/area_n, 100 g/area_p
    double *kn;                // per node: 100 g/area_n (0 at a root)
    double *D, *R;             // per position: rows handed between passes, global-scratch units
    double *DV;                // per position: v_parent - v_node of this step (global-scratch units)
};

struct FusedArgs {
    SlotDev slot[kMaxSlots];
    int n_slots;
    int has_syn;
    const int *tiles;          // (n_tiles + 1) rows of (1 + n_slots) ints
    int n_tiles;
    int row;                   // 1 + n_slots
    const long long *kdev;     // step counter in device memory
    int kofs;                  // k = *kdev + kofs
    int xcd_order;             // XCD-contiguous tile order (launch flag bit 0)
    int nontemporal;           // non-temporal SoA streams (launch flag bit 1)
    int *err;
    GlobDev g;
    NodesDev nd;
    int has_ext;               // a type only the extended instantiations handle (cabuf)
};

// Time-fused path: each workgroup stages one tile (its nodes and every
// instance on them) in LDS, advances it over `nsub` steps there, and writes
// it back once.
struct ResArgs {
    long long k0;              // step of the launch's first current update
    int nsub;                  // current updates (steps) in this launch
    int first_state;           // state update of step k0-1 before the first current update
    int last_state;            // state update at v_{k0+nsub} after the last one
};

// The arrays of a mechanism kind as the time-fused path stages them: STATEs,
// PARAMETERs (bit j of param_double: stored in FP64 in both precisions),
// the calcium current, the event stream id.  A compile-time copy of the
// kind table's shapes, checked against it on the host before every launch.
struct KindShape {
    int n_state, n_param, param_double, has_ica, has_gid;
};
__host__ __device__ constexpr KindShape kind_shape(int kind) {
    return kind == MECH_PAS       ? KindShape{0, 2, 0, 0, 0}
           : kind == MECH_HH      ? KindShape{3, 4, 0, 0, 0}
           : kind == MECH_IH      ? KindShape{1, 1, 0, 0, 0}
           : kind == MECH_CAHVA   ? KindShape{3, 1, 0, 1, 0}
           : kind == MECH_SYN     ? KindShape{4, 1, 1, 0, 1}
           : kind == MECH_KMARKOV ? KindShape{3, 1, 0, 0, 0}
           : kind == MECH_CAPUMP  ? KindShape{3, 1, 0, 1, 0}
           : kind == MECH_CABUF   ? KindShape{4, 1, 0, 1, 0}
                                  : KindShape{0, 0, 0, 0, 0};
}

__host__ __device__ inline size_t res_round8(size_t b) { return (b + 7) & ~(size_t)7; }

// LDS bytes of one slot's instance arrays in a tile of n of its instances
// (ss: bytes of a stored STATE): STATEs, PARAMETERs, ica, the tile-local
// node index, the event stream id.
__host__ __device__ inline size_t res_slot_bytes(int kind, int n, int ss) {
    const KindShape k = kind_shape(kind);
    const size_t nn = (size_t)n;
    size_t b = 0;
    for (int j = 0; j < k.n_state; ++j) b += res_round8(nn * ss);
    for (int j = 0; j < k.n_param; ++j) b += res_round8(nn * (((k.param_double >> j) & 1) ? 8 : ss));
    if (k.has_ica) b += res_round8(nn * ss);
    b += res_round8(nn * 4);
    if (k.has_gid) b += res_round8(nn * 4);
    return b;
}

// LDS 8-byte words per tile node: v, the rhs and d accumulators (two words
// each), 100/area (point processes), 1e-3 cm/dt (isolated) or the four clamp
// waveform parameters, and the shared calcium ion's cai and ica accumulator
// (two words); then an int spike counter per node and a 16-byte aligned
// table: 16 bytes per slot and 32 bytes of run ends.
__host__ __device__ inline int res_node_doubles(int vmode, bool has_syn, bool ion) {
    return 5 + (has_syn ? 1 : 0) + (vmode == MECH_V_CLAMP ? 4 : 1) + (ion ? 3 : 0);
}
__host__ __device__ inline size_t res_node_bytes(int nn, int vmode, bool has_syn, bool ion) {
    return 8 * (size_t)nn * res_node_doubles(vmode, has_syn, ion) + res_round8(4 * (size_t)nn) + 8 + 16 * (kMaxSlots + 2);
}

struct PlainArgs {
    SlotDev slot;
    long long k;
    int accumulate;            // unused by the state kernel
    int *err;
    GlobDev g;
    NodesDev nd;
    int atomic_scatter;        // one FP64 atomic per instance instead of the wave-segmented sum
    // per wave of the slot (ceil(n/64) entries): the node of a run that
    // began in an earlier wave, or -1, and that run's sums in this wave
    // (rhs, d, calcium current)
    int *carry_node;
    double *carry_val;
};

// Launchers (defined in mech_kernels.hip).  All return hipGetLastError().
hipError_t launch_fill(double *a, double *b, int n, hipStream_t s);
hipError_t launch_fill_int(int *a, int n, hipStream_t s);
hipError_t launch_set_k(long long *kdev, long long value, hipStream_t s);
hipError_t launch_bump_k(long long *kdev, long long by, hipStream_t s);
hipError_t launch_vclamp(const NodesDev &nd, double t, hipStream_t s);
hipError_t launch_visolated(const NodesDev &nd, const GlobDev &g, hipStream_t s);
hipError_t launch_init(bool fp32, const PlainArgs &a, hipStream_t s);
hipError_t launch_plain_cur(bool fp32, const PlainArgs &a, hipStream_t s);
hipError_t launch_plain_state(bool fp32, const PlainArgs &a, hipStream_t s);
hipError_t launch_stream(int op, int unroll, int flags, void *dst, const void *src, size_t bytes, int grid,
                         hipStream_t s);
hipError_t launch_cable(const CableDev &c, const NodesDev &nd, const GlobDev &g, hipStream_t s);
hipError_t cable_allow_lds(size_t bytes);
hipError_t launch_cable_coeffs(const CableDev &c, const double *area, int n_nodes, int n_edges, hipStream_t s);
hipError_t launch_fused(bool fp32, int phases, int vmode, const FusedArgs &a, int grid, int block, int tile_nodes,
                        hipStream_t s);
size_t fused_lds_bytes(int tile_nodes, bool ion);
hipError_t fused_allow_lds(size_t bytes);
hipError_t launch_resident(bool fp32, int vmode, const FusedArgs &a, const ResArgs &r, int grid, int block,
                           size_t lds_bytes, hipStream_t s);
hipError_t resident_allow_lds(size_t bytes);
hipError_t launch_ion_pool(const NodesDev &nd, const GlobDev &g, int *err, hipStream_t s);
hipError_t launch_ion_init(const NodesDev &nd, const GlobDev &g, hipStream_t s);

}  // namespace mech
