/*
 * dpsnn.h -- C ABI of the MI355X (gfx950) DPSNN simulation library, libdpsnn.so.
 *
 * The library simulates grids of cortical columns of leaky integrate-and-fire neurons
 * with calcium-driven spike-frequency adaptation, in 1 ms steps, the way the paper's
 * distributed simulator does (Pastorelli et al., arXiv:1511.09325): mixed time- and
 * event-driven (section 1) -- every neuron is integrated every step, and synaptic work
 * follows the spikes -- over columns of point neurons, 80 % excitatory, with
 * distance-decaying connectivity to the neighbouring columns and external Poisson
 * synapses (section 2, Methods).  The cost unit is the synaptic event: every current
 * reaching a neuron from a recurrent or an external synapse (section 3, Figure 2 caption).
 *
 * Conventions
 *   - All functions return DPSNN_OK (0) or a negative DPSNN_E* code; no C++ exception
 *     crosses the ABI.  After an error, sim_last_error() describes it.
 *   - "device" pointers are HIP device addresses (for example torch CUDA-tensor data
 *     pointers); "host" pointers are ordinary process memory.  The caller owns every
 *     buffer it passes; the library owns the memory behind a sim_t.
 *   - Work is enqueued on the HIP stream given at creation (NULL = the null stream).
 *     Functions marked "synchronises" wait for that stream.
 *   - A simulation holds one or more independent networks ("batched" form).  Neurons are
 *     numbered per network: column c = y*cols + x, neuron j = c*npc + k, k < n_exc
 *     excitatory.  Networks share the column recipe and neuron parameters and differ in
 *     grid shape, seed and external rate.
 *   - Synaptic input is integer fixed point (int32 at 2^-16 mV, wrap-around addition),
 *     so results do not depend on the order in which spikes are delivered.
 *   - Each call names the passage of the paper that defines what it computes, or says that
 *     it is part of the workload contract or of the library's own runtime (not in the paper).
 */
#ifndef DPSNN_H
#define DPSNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPSNN_OK 0
#define DPSNN_EINVAL (-1) /* bad argument or configuration */
#define DPSNN_ENOMEM (-2) /* device or host allocation failed */
#define DPSNN_EHIP (-3)   /* a HIP runtime call failed */
#define DPSNN_ESTATE (-4) /* call not valid in the current state */
#define DPSNN_ETRUNC (-5) /* an output buffer is too small (size needed is reported) */

/* Neuron model (section 2: LIF neurons with spike-frequency adaptation through calcium- and
 * sodium-dependent AHP currents; the Izhikevich RS/FS neurons of the earlier report). */
#define DPSNN_NEURON_LIF 0
#define DPSNN_NEURON_IZHIKEVICH 1

/* Connectivity kernel (section 2, Methods). */
#define DPSNN_CONN_EXP3X3 0 /* p_remote of the row over the 8 neighbours by exp(-r/decay_um) */
#define DPSNN_CONN_GAUSS 1  /* lateral_amp exp(-r^2/2 sigma^2) per pair over the cut stencil */

/* Spike delivery strategy. Both give bit-identical results. */
#define DPSNN_DELIVERY_AUTO 0
#define DPSNN_DELIVERY_ARRIVAL 1 /* per target column: gather arrivals, fused with the update */
#define DPSNN_DELIVERY_PUSH 2    /* per spike: scatter into a per-target delay ring (atomics) */

typedef struct sim sim_t;

/* One network of a simulation. */
typedef struct {
  int32_t rows, cols;  /* grid of columns, periodic (torus) */
  uint64_t seed;       /* Philox4x32-10 key of every random draw of this network */
  double ext_rate_hz;  /* rate of each external synapse */
} sim_net_t;

/* Configuration (copied by sim_create).  Units: mV, ms, Hz. */
typedef struct {
  /* column recipe (section 2, Methods) */
  int32_t npc;           /* neurons per column (the paper: 1240); 1 <= npc <= 4096 */
  int32_t n_exc;         /* excitatory neurons per column (the paper: 80 %) */
  double p_own;          /* pair connection probability inside a column */
  double p_remote;       /* share of a row spread over the 8 neighbour columns */
  double decay_um;       /* neighbour weight exp(-distance / decay_um) */
  double spacing_um;     /* column spacing (the paper: about 100 um) */
  int32_t d_min, d_max;  /* uniform integer delays in steps; 1 <= d_min <= d_max <= 32 */
  double we_mu, we_sigma; /* excitatory weights N(mu, sigma); |mu| + 6 sigma < 2 mV */
  double wi_mu, wi_sigma; /* inhibitory weights, mu < 0 */
  /* neuron (LIF with calcium-driven AHP) */
  double tau_m, theta, v_reset;
  int32_t t_ref;         /* refractory steps, 0..255 */
  double tau_ca, ca_inc, g_ahp, dt;
  /* external Poisson synapses */
  int32_t ext_syn;
  double j_ext;
  /* networks */
  int32_t n_nets;        /* >= 1 */
  const sim_net_t* nets; /* host array of n_nets */
  /* options */
  int32_t delivery;      /* DPSNN_DELIVERY_* */
  int32_t block;         /* threads per workgroup of the step kernels: 0 (auto), 64..1024 */
  int32_t tile_x, tile_y; /* arrival form: target columns per workgroup, 1..4 each; 0 0 = auto */
  int64_t record_steps;  /* spike raster: number of steps recorded from step 0 (0 = off) */
  int64_t raster_capacity; /* spike raster: capacity in spike ids */
  int32_t train_mode;    /* 1: float32 master weights, trajectory recording, sim_backward */
  int32_t ckpt_every;    /* train mode: checkpoint interval in steps (>= 1) */
  double surrogate_beta; /* train mode: slope of the fast-sigmoid surrogate, 1/mV (> 0) */
  /* neuron model variants (section 2 names the sodium-dependent AHP; neither variant is
   * parameterised in the paper).  LIF: a second AHP variable Na, V~ = ((P_m V - g_AHP dt Ca)
   * - g_na dt Na) + I, Na <- exp(-dt/tau_na) Na + na_inc s (off when g_na = 0).
   * Izhikevich (IEEE TNN 2003): two 0.5 ms Euler steps of v' = 0.04 v^2 + 5 v + 140 - u + I,
   * u <- u + a (b v - u), spike at v >= izh_vpeak, then v <- c, u <- u + d; excitatory
   * neurons take the _e parameters (RS), inhibitory ones the _i parameters (FS); no
   * refractory period; u is kept (and read by sim_read_state) where LIF keeps Ca; theta,
   * v_reset, t_ref, tau_m and the AHP fields are unused.  Train mode needs LIF with g_na = 0. */
  int32_t neuron_model;  /* DPSNN_NEURON_* */
  double tau_na, na_inc, g_na;
  double izh_a_e, izh_b_e, izh_c_e, izh_d_e;
  double izh_a_i, izh_b_i, izh_c_i, izh_d_i;
  double izh_vpeak;
  /* connectivity kernel (section 2, Methods: probability falling with the distance r between
   * column centres, cut at 1/1000).  DPSNN_CONN_EXP3X3 uses p_remote and decay_um over the
   * 3x3 stencil.  DPSNN_CONN_GAUSS gives every stencil offset other than the own column the
   * pair probability lateral_amp exp(-r^2 / (2 lateral_sigma_um^2)), the stencil being the
   * offsets whose exp(...) >= lateral_cutoff, at most 7x7 (the paper: sigma = the column
   * spacing, cut-off 1e-3, the 7x7 square minus its corners); p_remote and decay_um are
   * unused.  Offsets that wrap onto one column add their probabilities.  The arrival form
   * needs a native tiling whose parts hold at most 9 columns and whose source columns touch
   * at most 16 tiles (3x3, 3x2 or 2x2 tiles for the 7x7 stencil). */
  int32_t conn_kernel;   /* DPSNN_CONN_* */
  double lateral_amp, lateral_sigma_um, lateral_cutoff;
  /* spike-timing-dependent plasticity (sections 1-2 name it; off in the paper's runs, which
   * print no rule): with stdp = 1, the all-to-all pair rule with exponential traces on every
   * synapse of weight >= 0 (the excitatory ones).  Each pair of a spike's arrival at its
   * target (emission + delay) and a spike of the target changes the weight once: by
   * +a_plus exp(-(t_post - t_arr) / tau_plus) when the target's spike is not earlier than
   * the arrival, else by -a_minus exp(-(t_arr - t_post) / tau_minus); each change is
   * rounded to the 2^-14 mV weight unit where it is applied (depressions at arrival, after
   * the arriving spike has delivered its weight; potentiations after the update of the
   * step of the target's spike), and the weight is kept in [0, stdp_w_max].  A spike
   * delivers the weight it finds at arrival.  Needs the arrival form in the tiling of
   * creation, one step per gather, train_mode = 0, fewer than 2^24 neurons in at most 16000
   * columns and fewer than 2^35 synapse records.  Snapshots then also hold the weights and
   * traces. */
  int32_t stdp;          /* 0: off */
  double stdp_tau_plus, stdp_tau_minus; /* ms, > 0 */
  double stdp_a_plus, stdp_a_minus;     /* mV, >= 0 */
  double stdp_w_max;                    /* mV, 0 < w_max < 2 */
} sim_config_t;

/* Sizes of a created simulation. */
typedef struct {
  int32_t n_nets;
  int32_t n_cols;        /* all networks */
  int64_t n_neurons;     /* all networks */
  int64_t n_synapses;    /* all networks */
  int32_t ring_slots;    /* d_max + 1 */
  int64_t device_bytes;  /* device memory the library allocated and holds */
  int64_t caller_bytes;  /* device memory of the caller's buffers (sim_buffers_t) in use */
} sim_info_t;

/* Sizes of the device memory a configuration needs in the four regions a caller may own
 * (sim_query_sizes).  Every region is one contiguous buffer, 256-byte aligned; its arrays
 * sit at 256-byte aligned offsets in a fixed order:
 *   synapses  the synapse records (uint32, padding included, n_records + 4)
 *   index     the row starts (int64 [N+1]), the out-degrees (int32 [N]) and the per-part row
 *             index of the store
 *   state     V (float32 [N]) at state_v_offset, Ca (float32 [N]) at state_ca_offset and the
 *             refractory counters (uint8 [N]) at state_ref_offset, N = n_neurons, neurons of
 *             all networks in network order
 *   history   the spike history of the last d_max + 1 steps and its per-part entries
 * The library's other memory (column and tile tables, snapshots, the push ring, train-mode
 * buffers) it always allocates itself. */
typedef struct {
  int64_t n_neurons;       /* all networks */
  int64_t n_records;       /* records of the synapse store, group padding included */
  uint64_t synapse_bytes;
  uint64_t index_bytes;
  uint64_t state_bytes;
  uint64_t history_bytes;
  uint64_t state_v_offset, state_ca_offset, state_ref_offset;  /* bytes into the state region */
} sim_sizes_t;

/* Caller-owned device memory for sim_create (for example torch tensors): any of the four
 * regions may be NULL (the library then allocates it); a given region must be 256-byte
 * aligned and hold at least the bytes sim_query_sizes reports.  The caller keeps the buffers
 * alive until sim_destroy and must not touch them while the simulation runs, except to read
 * the state region between synchronising calls. */
typedef struct {
  void* synapses;
  uint64_t synapse_bytes;
  void* index;
  uint64_t index_bytes;
  void* state;
  uint64_t state_bytes;
  void* history;
  uint64_t history_bytes;
} sim_buffers_t;

/* Per-network counters since creation (or the last restore). */
typedef struct {
  int64_t steps;
  int64_t spikes;
  int64_t events_recurrent; /* outgoing synapses of every emitted spike */
  int64_t events_external;  /* external Poisson arrivals drawn */
  int64_t synapses_streamed; /* synapse records read by the delivery kernels */
  int64_t synapses_delivered; /* arrival form: records that fell into their reader's tile */
} sim_stats_t;

/* Paper section 2 (Methods) and Table 1: the network a configuration defines -- its grid
 * of columns, the connectivity that decides the size of the synapse store -- measured
 * without building it: the generator's count pass runs on the current device's null
 * stream, and the sizes of the four caller-ownable regions of sim_create come back in
 * *sizes.  DPSNN_EINVAL for a bad configuration (sim_last_error(NULL) tells why).
 * Synchronises. */
int sim_query_sizes(const sim_config_t* cfg, sim_sizes_t* sizes);

/* Paper section 2 (Methods), Table 1: build the networks on the device (connectivity,
 * delays, weights with integer delays) and set the initial state (V uniform on [0, v_reset),
 * Ca = 0, no pending input).
 * bufs: NULL, or caller-owned device buffers for some of the regions (sim_buffers_t).
 * hip_stream: a hipStream_t or NULL.  On success *out receives the handle; on failure it
 * is NULL and sim_last_error(NULL) tells why (DPSNN_EINVAL also when a caller buffer is
 * too small or misaligned).  Synchronises. */
int sim_create(const sim_config_t* cfg, const sim_buffers_t* bufs, void* hip_stream,
               sim_t** out);

/* Library runtime (not in the paper): release everything the handle holds; the caller's
 * buffers are left alone.  NULL is ignored. */
void sim_destroy(sim_t* sim);

/* Paper section 1: advance all networks by n_steps 1 ms steps of the mixed time- and
 * event-driven simulation (every neuron each step, synaptic work per spike).  Asynchronous.
 * A raster overflow is sticky and reported by the next synchronising call as DPSNN_ETRUNC.
 * In train mode the steps are launched one by one (graph_steps is not used) and the state
 * is checkpointed every ckpt_every steps. */
int sim_step(sim_t* sim, int64_t n_steps);

/* Library runtime (not in the paper): wait for the stream; returns a sticky error if one is
 * pending. */
int sim_sync(sim_t* sim);

/* Paper section 3 and Figure 2's caption (the spikes behind the synaptic events the paper
 * counts): recorded spikes of network `net` for steps [t0, t1): step_offsets (host,
 * t1-t0+1) and ids (host, network-local neuron ids, ascending within a step).  If ids_cap
 * is too small, returns DPSNN_ETRUNC with the needed count in *n_ids.  Synchronises. */
int sim_read_spikes(sim_t* sim, int32_t net, int64_t t0, int64_t t1, int64_t* step_offsets,
                    int32_t* ids, int64_t ids_cap, int64_t* n_ids);

/* sim_read_spikes for callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): same arguments, results and
 * errors, but no device or host allocation.  Its device scratch is a file-scope array of
 * 16 MiB per device, held until the process ends, which bounds one call to 24 bytes per step
 * of [t0, t1) plus 4 bytes per id returned (DPSNN_EINVAL beyond).  Every call on one device
 * shares that array, so calls that overlap on one device race.  Synchronises. */
int sim_read_spikes_static(sim_t* sim, int32_t net, int64_t t0, int64_t t1,
                           int64_t* step_offsets, int32_t* ids, int64_t ids_cap, int64_t* n_ids);

/* Workload contract (training; not in the paper, whose simulator has no gradients): go
 * back to the state at step 0 (the initial state) and start a new recorded window; counters
 * and per-column spike counts restart from zero.  Train mode only. */
int sim_rewind(sim_t* sim);

/* Paper section 2 (the per-column firing activity of the grid): mean firing rate of every
 * column since step 0 (or the last rewind), in Hz: R_c = 1000 * spikes_c / (npc * now * dt).
 * rates: device float32 [n_cols]. Asynchronous. */
int sim_column_rates(sim_t* sim, float* rates);

/* Workload contract (training; not in the paper): surrogate-gradient backward of the loss
 * L = (1/C) sum_c (R_c - R*_c)^2 between every column's mean rate since step 0 and its
 * target, through the recorded window [0, now) of train mode, for the paper's section 2
 * neuron (LIF with calcium-driven AHP).
 * target_rates: device float32 [n_cols of all networks], R*_c in Hz.
 * loss:         device float32 [1] (nullable): L.
 * grad_w, grad_tau_m, grad_g_ahp: as in sim_backward_rates.
 * Same costs, state and errors as sim_backward_rates.  Synchronises. */
int sim_backward(sim_t* sim, const float* target_rates, float* loss, float* grad_w,
                 double* grad_tau_m, double* grad_g_ahp);

/* Workload contract (training; not in the paper): sim_backward for any loss of the column
 * rates, given its gradient (for example from torch autograd).
 * grad_rates: device float32 [n_cols of all networks], dL/dR_c of each column's mean rate
 *             R_c = 1000 / (npc * T * dt) * spikes of column c (Hz).
 * grad_w:     device float32 [n_synapses], dL/dw in the canonical synapse order (per
 *             network, per source neuron, sorted by (delay, target)), w in mV.
 * grad_tau_m, grad_g_ahp: host doubles (nullable).
 * The reverse pass re-runs each checkpoint segment forward to record its trajectory (all
 * but the last, which the train-mode forward records as it steps, when nothing has
 * interrupted that recording), so it costs up to one forward plus the adjoint; afterwards
 * the state is the end state again.  The result does not depend on ckpt_every.
 * The adjoint (float32; float64 partial sums for the two scalars) follows the surrogate
 * recursion: nu = dL/dV~ = (1 - r)[lambda (1 - s) + e sigma'(V~ - theta)], sigma'(x) =
 * 1/(1 + beta|x|)^2, with lambda = dL/dV and e = dL/ds including the delayed synapses, whose
 * weights are the efficacies the forward delivered (rint(w 2^16) 2^-16 mV: the rounding is
 * passed straight through to the master weights).
 * Returns DPSNN_ESTATE if not in train mode, if nothing was recorded, or if the window was
 * broken (restore of another window, weight or parameter change after step 0; call
 * sim_rewind).  Synchronises. */
int sim_backward_rates(sim_t* sim, const float* grad_rates, float* grad_w, double* grad_tau_m,
                       double* grad_g_ahp);

/* Library runtime (not in the paper): error text of the last failing call on `sim`, or of
 * the last failing sim_create or sim_query_sizes of this thread when sim is NULL.  Never
 * NULL. */
const char* sim_last_error(const sim_t* sim);

/* Paper Table 1 (columns, neurons, synapses of a grid): sizes of a created simulation. */
int sim_get_info(const sim_t* sim, sim_info_t* info);

/* Paper section 3 and Figure 2's caption (the synaptic event: every current from a
 * recurrent or an external synapse): counters of network `net`.  Synchronises. */
int sim_get_stats(sim_t* sim, int32_t net, sim_stats_t* stats);

/* Library runtime (not in the paper): current step number (steps done).  Host-side, no
 * synchronisation. */
int64_t sim_now(const sim_t* sim);

/* Paper sections 1-2 (the neuron state and the delayed input of the step), a debug/test
 * view of network `net` (host buffers, n = neurons of the network):
 * v, ca (float32 [n]), ref (uint8 [n]), pend (int32 [ring_slots][n]) where pend[q][j] is
 * the recurrent input already emitted towards neuron j for step now+q (the delivery
 * strategy's internal form is converted to this view), na (float32 [n], the sodium AHP
 * variable; zeros when g_na = 0).  Any pointer may be NULL.
 * Synchronises. */
int sim_read_state(sim_t* sim, int32_t net, float* v, float* ca, uint8_t* ref, int32_t* pend,
                   float* na);

/* Paper section 2 (Methods: the synapses, their delays and weights), synapses of network
 * `net`, source neurons [i0, i1), in canonical order: row_ptr (host,
 * i1-i0+1, relative to the first), tgt (int32 network-local), dly (uint8), wq (int16, 2^-14
 * mV; with plasticity on, the weights as they are now).  Returns DPSNN_ETRUNC with row_ptr
 * filled if cap is short.  Synchronises. */
int sim_read_synapses(sim_t* sim, int32_t net, int64_t i0, int64_t i1, int64_t* row_ptr,
                      int32_t* tgt, uint8_t* dly, int16_t* wq, int64_t cap);

/* Library runtime (checkpoint/resume; not in the paper): snapshot slots, save or restore the
 * whole dynamic state (V, Ca, refractory counters,
 * pending input, step counter, event counters, per-column spike counts; with plasticity on
 * also the weights and the traces).  slot in [0, 64).
 * Asynchronous.  In train mode, restoring a state saved in another recorded window (before
 * the last sim_rewind, weight or parameter change) makes sim_backward fail until the next
 * sim_rewind; slot 63 is used by sim_autotune. */
int sim_save(sim_t* sim, int32_t slot);
int sim_restore(sim_t* sim, int32_t slot);

/* Workload contract (training; not in the paper): train mode's master weights (device
 * float32 [n_synapses], mV, canonical order) of the paper's section 2 synapses.  The
 * forward uses rint(w * 2^16) as int32 efficacy.  set copies in, get copies out; both are
 * asynchronous.  Initially the master weights are the generated int16 weights times 2^-14.
 * A set after step 0 of the recorded window breaks the window (see sim_backward). */
int sim_set_weights(sim_t* sim, const float* w);
int sim_get_weights(sim_t* sim, float* w);
/* Paper section 2 (the LIF neuron's membrane time constant and its calcium-driven AHP):
 * change tau_m and g_AHP (the constants are recomputed on the host; they reach the next
 * step, also under graph replay).  In train mode a change after step 0 of the recorded
 * window breaks the window (see sim_backward). */
int sim_set_params(sim_t* sim, double tau_m, double g_ahp);

/* Library runtime (not in the paper): launch configuration of the step: delivery strategy,
 * workgroup size and, for the arrival
 * form, the tile of target columns one workgroup owns (its LDS accumulators must fit in
 * 160 KB: gather_steps * tile_x * tile_y * npc * 4 bytes plus about 20 KB).  The synapse
 * store is split by the tiling chosen at creation; other tilings work but read more. */
typedef struct {
  int32_t delivery;  /* DPSNN_DELIVERY_ARRIVAL or DPSNN_DELIVERY_PUSH */
  int32_t block;     /* 64, 128, 256, 512 or 1024 (arrival form: the gathering steps; the
                        steps inside a gather window launch with at most 512 threads and one
                        accumulator, two workgroups per compute unit) */
  int32_t tile_x, tile_y;  /* 1..4 */
  int32_t graph_steps;     /* steps per captured HIP graph, replayed by sim_step; 0 = direct */
  int32_t gather_steps;    /* arrival form: steps whose input one pass over the spike history
                              gathers (adjacent delay groups read together), 1..8; 0 = the
                              largest that fits the LDS, at most 4 */
} sim_launch_t;

/* Library runtime: the launch configuration in use (gather_steps: the window in effect). */
int sim_get_launch(const sim_t* sim, sim_launch_t* launch);
/* Library runtime: change it between steps (synchronises); results are bit-identical for
 * every choice.  With plasticity on, only the workgroup size and graph_steps may change
 * (the delivery, the tiling and gather_steps 0 or 1 stay as they are); other requests are
 * DPSNN_EINVAL. */
int sim_set_launch(sim_t* sim, const sim_launch_t* launch);

/* Library runtime (determinism checks; not in the paper): order-independent 64-bit digest
 * of the dynamic state (V, Ca, refractory counters, spike
 * history).  Equal states give equal digests; used to check that launch configurations and
 * resumed runs agree bit for bit.  Synchronises. */
int sim_state_digest(sim_t* sim, uint64_t* digest);

/* Library runtime (not in the paper): the autotuner.  From the current state (kept in
 * snapshot slot 63), runs `window` steps with
 * each candidate launch configuration (delivery form, workgroup size, gather window, graph
 * chunk; the arrival form keeps the tiling of creation), timed with HIP events, checks that every candidate reaches the same state digest,
 * restores the state and keeps the fastest.  cache_path (nullable): a JSON-lines file of
 * earlier results keyed by the device and the simulation's shape; a hit skips the search.
 * best / best_ms_per_step (nullable) receive the choice.  DPSNN_ESTATE if two candidates
 * disagree.  Synchronises. */
int sim_autotune(sim_t* sim, int32_t window, const char* cache_path, sim_launch_t* best,
                 double* best_ms_per_step);

/* Library runtime (not in the paper): choose the arrival form's native tiling (the tile shape
 * the synapse store is split for, fixed at creation) by measurement.  For every shape of
 * 3x3, 3x2, 2x3, 2x2, 2x1, 1x2 and 1x1 that the configuration admits (that fits the LDS,
 * the stencil's part limits and the device memory), one at a time: the
 * simulation is created with that native tiling (cfg's tile fields and raster options are
 * replaced, everything else kept), steps `settle` untimed steps, then `window` steps timed
 * with HIP events on its stream, and is destroyed.  Every shape must reach the same state
 * digest (DPSNN_ESTATE otherwise).  tile_x, tile_y receive the fastest shape and
 * ms_per_step (nullable) its time per step.  Needs the device memory of one simulation at
 * a time; synchronises.  Errors (NULL pointers, settle < 0, window < 1, no admissible shape)
 * are reported by sim_last_error(NULL). */
int sim_tune_tiling(const sim_config_t* cfg, int32_t settle, int32_t window, int32_t* tile_x,
                    int32_t* tile_y, double* ms_per_step);

/* Paper section 3 (time per synaptic event, measured here per kernel): per-kernel device
 * time of the last sim_step call, measured with HIP events recorded on
 * the simulation's stream around every kernel launch while timing is on.  ms[0..2]: total
 * milliseconds of class 0 (the update kernel; in the arrival form it also gathers the
 * delivered input), class 1 (push delivery) and class 2 (raster recording); ms[3..5]: the
 * number of launches of each class.  n is the capacity of ms (up to 6 are written). */
int sim_set_timing(sim_t* sim, int32_t on);
int sim_get_timing(sim_t* sim, double* ms, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
