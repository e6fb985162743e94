/*
 * mech.h -- C ABI of the MI355X mechanism-kernel library (libmech.so).
 *
 * The library advances the membrane mechanisms of a compartmental neuron
 * model by one or many fixed timesteps on one GPU.  Its two kernels are the
 * ones the paper's NMODL compiler generates and accelerates (section 1 and
 * section 8, "current update" and "state update"):
 *
 *   nrn_cur   (mech_cur)   -- BREAKPOINT block (section 3): gather the node
 *             voltage v through each instance's node index, evaluate the
 *             channel or synapse current i(v) with every STATE frozen, its
 *             conductance g = (i(v+dv) - i(v))/dv by finite difference (the
 *             default run-time approximation named in section 5.2), and
 *             reduce rhs[node] -= s*i, d[node] += s*g;
 *   nrn_state (mech_state) -- DERIVATIVE + SOLVE ... METHOD cnexp (sections 3
 *             and 5.2): every gating or decay STATE x' = (x_inf - x)/tau is
 *             advanced by its analytic solution with coefficients held
 *             constant over the step.
 *
 * Mechanism types (section 3: SUFFIX = density mechanism, POINT_PROCESS =
 * synapse; RANGE / PARAMETER / ASSIGNED / STATE variables):
 *   MECH_PAS    density, i = g (v - e)                      params g, e
 *   MECH_HH     density, Hodgkin-Huxley Na/K/leak           params gnabar, gkbar, gl, el
 *                                                           states m, h, n
 *   MECH_IH     density, one hyperpolarisation-activated gate, i = gbar m (v - eh)
 *                                                           params gbar; states m
 *   MECH_CAHVA  density, m^2 h calcium current with Nernst eca and a
 *               submembrane calcium pool (cai relaxes to cai0 with tau_ca)
 *                                                           params gbar; states m, h, cai
 *   MECH_SYN    point process, double-exponential AMPA + NMDA conductance
 *               with Mg block; a NET_RECEIVE-style event of weight w adds w*f
 *               to both rise (A) and decay (B) states of each receptor
 *                                                           params weight (nS)
 *                                                           states A_ampa, B_ampa, A_nmda, B_nmda
 *   MECH_KMARKOV density, three-state potassium scheme C1 <-> C2 <-> O with
 *               the Hodgkin-Huxley n rates (2a, b, a, 2b), i = gbar O (v - ek),
 *               advanced by implicit Euler: one 3x3 linear solve per instance
 *               (the sparse method of section 5.2)      params gbar; states C1, C2, O
 *   MECH_CAPUMP density, Ca-HVA gates with a calcium pool emptied by a
 *               saturable pump, vmax (c/(c+kp) - cai0/(cai0+kp)); the pool's
 *               implicit Euler equation is solved by Newton's method with the
 *               analytic derivative (derivimplicit, section 5.2)
 *                                                           params gbar; states m, h, cai
 *   MECH_CABUF  density, Ca-HVA gates with free calcium cai and calcium
 *               bound to a buffer, cab (binding kon cai (btot - cab) -
 *               koff cab, cai relaxing to cai0 with tau_ca); the pool's two
 *               coupled implicit Euler equations are solved by Newton's
 *               method on the 2x2 system (derivimplicit, section 5.2)
 *                                                           params gbar; states m, h, cai, cab
 *
 * Units: mV, ms, mA/cm2 and S/cm2 for density mechanisms, nA and uS for the
 * synapse (scaled by 100/area into the node vectors), um2, uF/cm2, mM, degC,
 * Hz; synaptic weights and states in nS.
 *
 * Precision (MECH_FP64 / MECH_FP32_MIXED): FP64 keeps every variable in
 * double, as the paper's generated code does (section 4.3).  FP32_MIXED
 * stores STATEs and every RANGE PARAMETER read each step in float
 * (conductances and per-instance reversal potentials such as pas e and hh
 * el; a float reversal potential moves by at most about 5e-6 mV) and
 * computes rates and the state update in float with the hardware
 * exponential.  v, the global reversal potentials (ena, ek, eh, e_syn), the
 * driving force v - e (formed in double from the stored e), the Nernst
 * potential, the Mg block, the finite difference and the rhs/d reduction
 * stay in double; synaptic weights, read only on an event, stay in double.
 *
 * Memory ownership: the caller allocates one device buffer of
 * mech_required_bytes() bytes and passes it to mech_alloc(); the library
 * carves every instance array out of it and never frees it.  Node vectors
 * (v, rhs, d, area, cm, clamp waveform) are caller-owned device arrays bound
 * by pointer.  Host arrays passed to mech_set_* are copied before return.
 * The library may reorder instances internally (sorted by node); every host
 * array in or out is in the caller's instance order.
 *
 * Streams: all device work is enqueued on the stream given to mech_alloc
 * and is asynchronous, except mech_get_state, mech_set_state,
 * mech_set_params, mech_spike_counts, mech_sync and mech_autotune, which
 * return after the stream has drained.
 *
 * Errors: every call returns MECH_OK (0) or a negative MECH_ERR_* code and
 * records a message for mech_last_error().  No call aborts and no C++
 * exception crosses this interface.  A context is not thread safe; distinct
 * contexts are independent.
 */
#ifndef MECH_H
#define MECH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MECH_OK = 0,
    MECH_ERR_INVAL = -1,       /* null pointer, bad kind / name / size / mode   */
    MECH_ERR_RANGE = -2,       /* node index outside [0, n_nodes)               */
    MECH_ERR_NOMEM = -3,       /* device buffer smaller than required           */
    MECH_ERR_STATE = -4,       /* call order (e.g. a step before mech_bind_nodes) */
    MECH_ERR_HIP = -5,         /* HIP runtime error, message in mech_last_error */
    MECH_ERR_NONFINITE = -6    /* a kernel produced a non-finite STATE          */
};

enum {
    MECH_PAS = 0, MECH_HH = 1, MECH_IH = 2, MECH_CAHVA = 3, MECH_SYN = 4, MECH_KMARKOV = 5, MECH_CAPUMP = 6,
    MECH_CABUF = 7
};
enum { MECH_FP64 = 0, MECH_FP32_MIXED = 1 };
/* voltage provision between the current and the state update of a step
 * (section 8, Table 3 "Other"):
 *   EXTERNAL  v is left as bound (the caller owns it);
 *   CLAMP     v[n] = off[n] + amp[n] sin(2 pi freq[n] t 1e-3 + phase[n]),
 *             t in ms, freq in Hz;
 *   ISOLATED  every node is an isolated compartment advanced by backward
 *             Euler, v += rhs/(1e-3 cm/dt + d), and an upward crossing of
 *             vthresh increments the node's spike count;
 *   CABLE     the nodes form trees (cells, mech_bind_cable) coupled by axial
 *             conductances: backward Euler of the cable equation linearised
 *             with rhs and d, (1e-3 cm/dt + d_n) dv_n + sum_j k_nj (dv_n -
 *             dv_j) = rhs_n + sum_j k_nj (v_j - v_n), k_nj = 100 g_nj/area_n,
 *             solved by Hines elimination; spikes as in ISOLATED.            */
enum { MECH_V_EXTERNAL = 0, MECH_V_CLAMP = 1, MECH_V_ISOLATED = 2, MECH_V_CABLE = 3 };
/* PLAIN: per step, one launch per mechanism type for the current update,
 *        one for the voltage, one per type for the state update, issued
 *        eagerly (the paper's per-mechanism kernel structure);
 * BATCHED: per step one fused launch over a table of node tiles that runs
 *        state(k-1), events(k) and cur(k) of every type and provides the
 *        next voltage, with chunks of steps replayed from a HIP graph.  Each
 *        node's rhs, d (and calcium current) is summed in fixed point with
 *        resolution 2^-67 (each contribution rounded to a multiple of 2^-67,
 *        exactly when its magnitude is >= 2^-15) and rounded to double
 *        once, so the result does not depend on the order in which
 *        contributions arrive: runs and launch shapes give the same bits;
 * RESIDENT: time-fused.  The BATCHED path's tiles, but each workgroup keeps
 *        its tile (node data and every instance array) in LDS for up to
 *        mech_set_resident_steps() steps and writes STATEs back once, so
 *        STATEs do not cross HBM every step.  Same per-step arithmetic and
 *        node sums as BATCHED (FP64: the same bits).  CLAMP and
 *        ISOLATED modes only (MECH_ERR_INVAL otherwise); every tile must fit
 *        the device's LDS per workgroup (160 KiB on gfx950; MECH_ERR_STATE
 *        otherwise: lower tile_instances / tile_nodes with
 *        mech_set_launch).  Between launches rhs/d are not written, only
 *        after the last step, which is what mech_step returns.              */
enum { MECH_PATH_PLAIN = 0, MECH_PATH_BATCHED = 1, MECH_PATH_RESIDENT = 2 };

typedef struct mech_ctx mech_ctx;

/* One mechanism type and its instances.  node_index (host, int32, count
 * entries, values in [0, n_nodes)) gives each instance's node; several
 * instances may share a node and the order is free.                       */
typedef struct {
    int32_t kind;
    int64_t count;
    const int32_t *node_index;
} mech_type_desc;

/* Bytes of the device buffer mech_alloc needs for these types (256-byte
 * aligned arrays, each padded to a multiple of 64 instances).             */
int mech_required_bytes(int64_t n_nodes, const mech_type_desc *types, int n_types, int prec,
                        size_t *out_bytes);

/* Create a context.  Validates every node index on the host (MECH_ERR_RANGE),
 * sorts instances by node (stable), carves the device buffer `dev_buf` of
 * `dev_bytes` bytes (MECH_ERR_NOMEM if short), uploads the index arrays and
 * the tile table, and sets every parameter to its default and every global
 * to its default.  `hip_stream` is a hipStream_t (NULL: the null stream).
 * At most 8 types; each count < 2^31; at most 2^19 instances (all types
 * together) on one node (MECH_ERR_INVAL), the bound of the fused paths'
 * fixed-point node sums.                                                  */
int mech_alloc(mech_ctx **out, int64_t n_nodes, const mech_type_desc *types, int n_types, int prec,
               void *dev_buf, size_t dev_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): mech_alloc with
 * the device buffer taken from a static area of the library instead of the
 * caller, 64 MiB on each device (held until the process ends).  Same
 * arguments, checks and results as mech_alloc otherwise; the context then
 * behaves as one made by mech_alloc (the caller still binds its node
 * vectors).  Allocates no device memory.  One live context per device:
 * MECH_ERR_STATE while another static context on the current device has not
 * been freed (mech_free releases the area, whose contents then stay until
 * the next mech_alloc_static overwrites them); MECH_ERR_NOMEM when
 * mech_required_bytes exceeds the area.  Calls from several host threads
 * are serialised; work of one static context on several streams races as
 * for any context.                                                         */
int mech_alloc_static(mech_ctx **out, int64_t n_nodes, const mech_type_desc *types, int n_types, int prec,
                      void *hip_stream);

/* Bind caller-owned device node vectors (double, n_nodes each).  v, rhs, d
 * are required; area is required if a MECH_SYN type exists; cm is required
 * for MECH_V_ISOLATED (may be NULL otherwise).                             */
int mech_bind_nodes(mech_ctx *ctx, double *v, double *rhs, double *d, const double *area,
                    const double *cm);

/* Bytes of the device buffer the cell trees of MECH_V_CABLE need, from the
 * host parent array (int32, n_nodes entries) and the unit_nodes that
 * mech_bind_cable will be given, for the current device.                   */
int mech_cable_required_bytes(int64_t n_nodes, const int32_t *parent, int32_t unit_nodes,
                              size_t *out_bytes);

/* Bind the cell trees for MECH_V_CABLE.  parent (host, int32[n_nodes]):
 * the parent of each node, -1 for a cell's root, with parent[n] < n (Hines
 * order) and every cell a contiguous node range that starts at its root
 * (MECH_ERR_INVAL otherwise).  g_axial (device, double[n_nodes], caller
 * owned): the axial conductance in uS between node n and its parent.
 * unit_nodes bounds the nodes one workgroup solves together in LDS (44 B
 * per node): 0 takes the library's default of 1024, a value above the
 * device's LDS capacity (3537 nodes on gfx950) is reduced to it, a
 * negative one is MECH_ERR_INVAL.  Any bound gives the same elimination up
 * to rounding; it only changes how cells are cut.  A cell larger than the bound is cut into subtrees that
 * fit and a trunk, which is solved in global memory if it is still too
 * large (a long unbranched cell).  The library builds the elimination
 * schedules into dev_buf (dev_bytes >=
 * mech_cable_required_bytes, 256-byte aligned, caller owned, MECH_ERR_NOMEM
 * if short) and computes the coupling coefficients 100 g/area from the
 * bound area and g_axial, so area (mech_bind_nodes, MECH_ERR_STATE if not
 * bound) and g_axial must hold their values at this call; bind again after
 * changing either.  cm is read every step.                                 */
int mech_bind_cable(mech_ctx *ctx, const int32_t *parent, const double *g_axial, int32_t unit_nodes,
                    void *dev_buf, size_t dev_bytes);

/* The cut of the cell trees that mech_bind_cable makes for this parent
 * array and unit_nodes on the current device, on the host only (no device
 * memory is touched), for inspection and tests.  sizes (int32[14])
 * receives the lengths of the plan's arrays, in this order: parent,
 * pos_node, pos_par, pos_src (per position: its node, the position of its
 * parent's row in the same unit or -1, for a ghost the piece root's own
 * position else -1), elim_n, elim_p (edge records: child and parent
 * position, a root paired with itself), elim_ptr (height boundaries),
 * unit_pos, unit_elim (per unit: position range, range into elim_ptr),
 * unit_mode (0 whole cells, 1 subtrees of a cut cell, 2 its trunk), and
 * the launch lists up, top (in LDS), top in global memory, down.  If buf is
 * not NULL the arrays are written back to back into it (int32, buf_len
 * entries; MECH_ERR_NOMEM if short).                                        */
int mech_cable_plan(int64_t n_nodes, const int32_t *parent, int32_t unit_nodes, int32_t *sizes,
                    int32_t *buf, int64_t buf_len);

/* Bind the clamp waveform (device, double, n_nodes each) for MECH_V_CLAMP. */
int mech_bind_clamp(mech_ctx *ctx, const double *off, const double *amp, const double *freq_hz,
                    const double *phase);

/* Set the RANGE parameter `name` of type slot `type_slot` from host memory:
 * n == 1 broadcasts one value, n == count gives one value per instance in the
 * caller's order.  Names: pas g,e; hh gnabar,gkbar,gl,el; ih gbar;
 * cahva gbar; syn weight; kmarkov gbar; capump gbar; cabuf gbar.          */
int mech_set_params(mech_ctx *ctx, int type_slot, const char *name, const double *host_vals, int64_t n);

/* Set a global: celsius, ena, ek, eh, cao, cai0, tau_ca, ca_gamma, ca_depth,
 * e_syn, mg, tau_r_ampa, tau_d_ampa, tau_r_nmda, tau_d_nmda, event_rate_hz,
 * event_seed (an integer below 2^53), vthresh, fd_dv, and the two variants
 * of section 5.2 (0 or 1, default 0):
 *   analytic_conductance  g = di/dv in closed form (the CONDUCTANCE
 *                         statement) instead of the finite difference;
 *   pade_cnexp            every cnexp factor exp(-dt/tau) replaced by its
 *                         (1,1) Pade approximant (1 - y/2)/(1 + y/2),
 *                         y = dt/tau (requires y < 2 to keep gates in
 *                         [0, 1]);
 * the pump of MECH_CAPUMP: pump_vmax (mM/ms), pump_kp (mM); the buffer of
 * MECH_CABUF: buf_total (mM), buf_kon (1/(mM ms)), buf_koff (1/ms);
 * newton_iters (1..16 Newton steps per implicit Euler step, default 4);
 * and shared_ca (0 or 1, default 0): calcium as a per-node ion, the USEION
 * dependency between mechanisms (section 3).  Every MECH_CAHVA, MECH_CAPUMP
 * and MECH_CABUF instance then reads its node's cai and adds its calcium
 * current to the node's total ica; one pool per node relaxes by the linear
 * pool law, cai_inf = cai0 - kappa tau_ca ica with time constant tau_ca,
 * from that total; the instances' own pools (cabuf's cab too) are left
 * untouched.  Needs a
 * calcium type (MECH_ERR_STATE otherwise); set it before mech_init, which
 * sets every node's cai to cai0.  The node arrays are read with
 * mech_get_state(ctx, -1, "cai" or "ica", ...).  Changing a global drops
 * the captured step graphs (rebuilt on the next batched step).             */
int mech_set_global(mech_ctx *ctx, const char *name, double value);

/* INITIAL (section 3): every gate at its steady state x_inf(v) at the bound
 * v, synapse states 0, cai = cai0 (each instance's and each node's), ica =
 * 0; spike counts 0.                                                       */
int mech_init(mech_ctx *ctx);

/* Current update of step k (t = k*dt): synapse events of step k, then
 * rhs[n] = -sum s*i, d[n] = sum s*g over every instance at node n
 * (accumulate != 0 adds to the existing rhs/d instead of overwriting).    */
int mech_cur(mech_ctx *ctx, int64_t k, double dt, int accumulate);

/* State update over one step of length dt at the bound v.                 */
int mech_state(mech_ctx *ctx, double dt);

/* Steps k0 .. k0+nsteps-1, each: events(k), cur at v_k, voltage provision
 * (vmode) to v_{k+1}, state at v_{k+1}.  In MECH_V_CLAMP mode v is set to
 * the clamp value at t_{k0} first.  On return (asynchronously) v holds
 * v_{k0+nsteps}, rhs/d hold the last step's current update and every STATE
 * is at t_{k0+nsteps}.                                                     */
int mech_step(mech_ctx *ctx, int64_t nsteps, int64_t k0, double dt, int vmode, int path);

/* Launch shape of the BATCHED path: threads per block (64..1024, multiple
 * of 64), tile work budget in instances (>= block), node span per tile
 * (64..2048), blocks per CU of a persistent grid (0: one block per tile)
 * and flags (MECH_LAUNCH_XCD_ORDER: consecutive tiles on the same XCD, so
 * the cache lines two neighbouring tiles share stay in one L2;
 * MECH_LAUNCH_NONTEMPORAL: instance arrays streamed with the non-temporal
 * hint, as they are touched once per step; MECH_LAUNCH_PLAIN_ATOMIC: the
 * PLAIN path's current update scatters one FP64 atomic per instance instead
 * of the wave-segmented per-node sum, for comparison).  Rebuilds
 * the tile table.  BATCHED and RESIDENT results do not depend on the shape
 * (their node sums are order-independent); PLAIN's rhs/d differ from one
 * run to the next by the rounding order of its atomics.                    */
enum { MECH_LAUNCH_XCD_ORDER = 1, MECH_LAUNCH_NONTEMPORAL = 2, MECH_LAUNCH_PLAIN_ATOMIC = 4 };
int mech_set_launch(mech_ctx *ctx, int block, int tile_instances, int tile_nodes, int blocks_per_cu,
                    int flags);
int mech_get_launch(const mech_ctx *ctx, int *block, int *tile_instances, int *tile_nodes,
                    int *blocks_per_cu, int *flags);

/* Steps per launch of the RESIDENT path (1..4096, default 64): STATEs
 * cross HBM once per launch.                                              */
int mech_set_resident_steps(mech_ctx *ctx, int steps_per_launch);

/* Time every candidate launch shape of the BATCHED path on `nsteps` steps
 * (HIP events, median of `reps`), time the four fastest again on 4 nsteps
 * steps (median of 2 reps), then tile sizes from 10/16 to 20/16 of the
 * fastest one's, keep the fastest, and return its ms per step.  STATEs, v, rhs, d, spike counts and the per-node calcium ion are
 * saved before and restored after, so the call has no visible effect
 * besides the chosen shape.                                                */
int mech_autotune(mech_ctx *ctx, double dt, int vmode, int nsteps, int reps, double *best_ms_per_step);

/* The same for the RESIDENT path (with the same second round and tile
 * refinement): launch shapes whose tiles fit the LDS of a workgroup, each
 * timed over `nsteps` steps (at most the steps per launch set by
 * mech_set_resident_steps per launch).  CLAMP and ISOLATED modes only.    */
int mech_autotune_resident(mech_ctx *ctx, double dt, int vmode, int nsteps, int reps, double *best_ms_per_step);

/* Copy STATE `name` (or "ica" for Ca-HVA, capump and cabuf) of type slot `type_slot` to /
 * from host doubles in the caller's instance order; n must equal count.
 * type_slot -1 names the per-node calcium ion instead: "cai" (mM) or "ica"
 * (mA/cm2, the last current update's total), n == n_nodes, present when a
 * calcium type exists (MECH_ERR_INVAL otherwise).                          */
int mech_get_state(mech_ctx *ctx, int type_slot, const char *name, double *host_out, int64_t n);
int mech_set_state(mech_ctx *ctx, int type_slot, const char *name, const double *host_in, int64_t n);

/* Spike counts per node (ISOLATED mode) to host int32[n_nodes].            */
int mech_spike_counts(mech_ctx *ctx, int32_t *host_out, int64_t n_nodes);

/* Drain the stream and report asynchronous errors (MECH_ERR_NONFINITE when
 * a kernel stored a non-finite STATE since the last call; the flag clears). */
int mech_sync(mech_ctx *ctx);

/* Number of tiles of the BATCHED path and the instance count of slot s.   */
int mech_info(const mech_ctx *ctx, int64_t *n_tiles, int64_t *max_tile_nodes);

/* Measurement aid (not part of a timestep): stream `bytes` (a multiple of
 * 16; device pointers, 16-byte aligned) with blocks_per_cu * n_CU blocks of
 * 256 threads on `hip_stream`, each thread keeping `unroll` (1, 2, 4, 8)
 * independent accesses in flight:
 *   op 0 copies src to dst;
 *   op 1 reads src (dst receives at most 16 bytes);
 *   op 2 writes dst;
 *   op 3 reads src[0, bytes) and src[bytes, 2 bytes) and writes their xor
 *        to dst (two reads per write, the STREAM-triad mix);
 *   op 4 reads src[0, bytes) in the even workgroups and writes dst[0, bytes)
 *        in the odd ones (read and write streams from different waves);
 *   op 5 treats dst[0, bytes) as seven FP64 arrays of n = bytes / 56
 *        elements (n a multiple of 256; src unused), reads all seven and
 *        rewrites the first three, the access shape of a Hodgkin-Huxley
 *        slot's STATEs and PARAMETERs (HBM traffic 10/7 bytes);
 *   op 6 treats dst[0, bytes) as twenty FP64 arrays of n = bytes / 160
 *        elements (n a multiple of 2048; src unused) in four groups of five,
 *        two of each group rewritten, streamed in tiles of 2048 elements
 *        dealt round-robin to the workgroups, group after group within a
 *        tile (the fused kernel's pattern; HBM traffic 28/20 bytes).
 * `flags` (bitwise or of MECH_PROBE_*): non-temporal hint on the loads or
 * on the stores, 8-byte instead of 16-byte accesses, one contiguous chunk
 * per workgroup instead of the grid-stride mapping, and for op 5 the seven
 * arrays interleaved in blocks of 256 elements instead of laid end to end,
 * or (TILED) tiles of 2048 elements dealt round-robin to the workgroups;
 * for op 6 AOSOA stores each tile's twenty arrays contiguously.
 * The streaming HBM ceilings the mechanism kernels are compared with.
 * Asynchronous.                                                            */
#define MECH_PROBE_NT_LOAD 1
#define MECH_PROBE_NT_STORE 2
#define MECH_PROBE_8B 4
#define MECH_PROBE_CHUNKED 8
#define MECH_PROBE_AOSOA 16
#define MECH_PROBE_TILED 32
int mech_probe_stream(int op, int unroll, int blocks_per_cu, int flags, void *dst, const void *src, size_t bytes,
                      void *hip_stream);

const char *mech_last_error(const mech_ctx *ctx);
const char *mech_strerror(int code);
void mech_free(mech_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
