/*
 * dpsnn_oracle.h -- plain, slow CPU oracle of the DPSNN per-1 ms simulation step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or
 * call this code; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP path.
 *
 * What it computes (paper sections cited per function in dpsnn_oracle.c):
 *   - the synthetic network: a torus grid of cortical columns of point neurons,
 *     80 % excitatory / 20 % inhibitory, distance-decaying column-to-column
 *     connectivity, integer delays (paper section 2, Methods);
 *   - the mixed time/event-driven step (paper section 1): every neuron is
 *     integrated every 1 ms step (LIF with calcium-driven spike-frequency
 *     adaptation, paper section 2), and every spike is fanned out through its
 *     outgoing synapses into a per-target delay ring of integer fixed-point input;
 *   - the counts behind the paper's cost unit, the synaptic event, which covers
 *     both recurrent and external synapses (paper section 3, Figure 2 caption).
 *
 * Arithmetic contract (shared reading with the HIP path, written independently):
 *   - synaptic input is summed as int32 at 2^-16 mV with wrap-around, so sums are
 *     order independent;
 *   - neuron state is float32, every operation rounded to nearest, evaluated in a
 *     fixed order with no fused multiply-add (build with -ffp-contract=off);
 *   - random numbers come from Philox4x32-10 (Salmon et al., SC'11), keyed by the
 *     64-bit network seed and addressed by a 4-word counter whose last word names
 *     the purpose (ORC_STREAM_*).
 */
#ifndef DPSNN_ORACLE_H
#define DPSNN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_STREAM_SYN = 1,  /* counter (j, i, sub, 1): pair i->j connection, delay, weight */
  ORC_STREAM_EXT = 2,  /* counter (j/4, u, 0, 2), word j%4: external Poisson count of neuron j at step u */
  ORC_STREAM_INIT = 3  /* counter (j, 0, 0, 3):   initial membrane potential of neuron j */
};

typedef struct {
  int32_t rows, cols;   /* grid of columns, periodic in both directions */
  int32_t npc;          /* neurons per column */
  int32_t n_exc;        /* excitatory neurons per column: local index k < n_exc */
  uint64_t seed;        /* Philox key */
  double p_own;         /* connection probability of a pair in the same column */
  double p_remote;      /* share of a row spread over the 8 neighbour columns */
  double decay_um;      /* length scale of the exponential decay over distance */
  double spacing_um;    /* column spacing */
  int32_t d_min, d_max; /* integer delays in steps, 1 <= d_min <= d_max */
  double we_mu, we_sigma; /* excitatory weight, mV */
  double wi_mu, wi_sigma; /* inhibitory weight, mV (mu < 0) */
  double tau_m;         /* membrane time constant, ms */
  double theta;         /* threshold, mV */
  double v_reset;       /* reset potential, mV */
  int32_t t_ref;        /* refractory period, steps */
  double tau_ca;        /* calcium time constant, ms */
  double ca_inc;        /* calcium increment per spike */
  double g_ahp;         /* AHP conductance: mV per unit calcium per ms */
  double dt;            /* step, ms */
  double ext_rate_hz;   /* rate of each external synapse */
  int32_t ext_syn;      /* external synapses per neuron */
  double j_ext;         /* external synaptic efficacy, mV */
  /* neuron model variants (paper section 2: spike-frequency adaptation through calcium- and
   * sodium-dependent AHP currents; the earlier report's Izhikevich RS/FS neurons) */
  int32_t neuron_model; /* ORC_NEURON_LIF or ORC_NEURON_IZHIKEVICH */
  double tau_na;        /* LIF: time constant of the sodium-dependent AHP variable, ms */
  double na_inc;        /* LIF: its increment per spike */
  double g_na;          /* LIF: its conductance, mV per unit per ms (0: one AHP variable) */
  double izh_a_e, izh_b_e, izh_c_e, izh_d_e;  /* Izhikevich, excitatory neurons (RS) */
  double izh_a_i, izh_b_i, izh_c_i, izh_d_i;  /* Izhikevich, inhibitory neurons (FS) */
  double izh_vpeak;     /* Izhikevich spike cut-off, mV */
  /* connectivity kernel (paper section 2, Methods): ORC_CONN_EXP3X3 spreads p_remote over the
   * 8 neighbours by exp(-r / decay_um); ORC_CONN_GAUSS gives every stencil offset at column
   * distance r the pair probability lateral_amp exp(-r^2 / (2 lateral_sigma_um^2)), the
   * stencil being the offsets whose exp(-r^2 / (2 sigma^2)) >= lateral_cutoff (the paper's
   * 1/1000 cut-off: the 7x7 square minus its corners for sigma = the column spacing) */
  int32_t conn_kernel;
  double lateral_amp, lateral_sigma_um, lateral_cutoff;
  /* spike-timing-dependent plasticity (paper sections 1-2 name it; off in its runs): an
   * all-to-all pair rule with exponential traces on the synapses of excitatory sources
   * (see orc_sim_step) */
  int32_t stdp;         /* 0: off */
  double stdp_tau_plus, stdp_tau_minus;  /* trace time constants, ms */
  double stdp_a_plus, stdp_a_minus;      /* weight change per unit trace, mV */
  double stdp_w_max;                     /* upper weight bound, mV */
} orc_config_t;

enum { ORC_NEURON_LIF = 0, ORC_NEURON_IZHIKEVICH = 1 };
enum { ORC_CONN_EXP3X3 = 0, ORC_CONN_GAUSS = 1 };

/* Half-width of the connectivity stencil in columns (1 for the 3x3 kernel). */
int32_t orc_stencil_radius(const orc_config_t* cfg);

/* Host threads of the loops over independent rows and neurons (OpenMP); results do not
 * depend on the thread count. */
void orc_set_threads(int32_t n);
int32_t orc_threads(void);

/* Philox4x32-10 block function. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Pair connection probability from source column to target column. */
double orc_column_probability(const orc_config_t* cfg, int32_t src_col, int32_t tgt_col);

/* Decide pair i->j directly; returns 1 and fills delay / 2^-14 mV weight if connected. */
int orc_pair(const orc_config_t* cfg, int64_t i, int64_t j, int32_t* delay, int16_t* wq);

/* Outgoing row of neuron i sorted by (delay, target); returns its length or -1 if cap is short. */
int64_t orc_row(const orc_config_t* cfg, int64_t i, int32_t* tgt, uint8_t* dly, int16_t* wq,
                int64_t cap);

/* Whole network as CSR; row_ptr has n+1 entries. Returns total synapses or -1 if cap is short. */
int64_t orc_network(const orc_config_t* cfg, int64_t* row_ptr, int32_t* tgt, uint8_t* dly,
                    int16_t* wq, int64_t cap);

/* Inverse-CDF thresholds of Poisson(lam) as 64-bit integers: tab[k] = min(floor(F(k) 2^32), 2^32). */
void orc_poisson_table(double lam, uint64_t tab[63]);
/* Count drawn from a 32-bit uniform: number of k in [0,63) with tab[k] <= x. */
int32_t orc_poisson_count(const uint64_t tab[63], uint32_t x);

/* External counts n_j(u) of neurons j0 .. j0+n-1 at step u. */
void orc_ext_counts(const orc_config_t* cfg, int64_t u, int64_t j0, int64_t n, int32_t* out);

/* Update one neuron at step u from its state and recurrent input (2^-16 mV), drawing its
 * external count; returns the spike flag.  Same arithmetic as a simulation step.  ca holds
 * the Izhikevich recovery variable u for that model; na (the sodium-dependent AHP variable)
 * may be NULL when g_na = 0. */
int orc_neuron_update(const orc_config_t* cfg, int64_t j, int64_t u, int32_t rec_input, float* v,
                      float* ca, uint8_t* ref, float* na);

/* orc_neuron_update for neurons j0 .. j0+n-1 at step u (arrays of n, updated in place;
 * spk receives the spike flags; na may be NULL when g_na = 0). */
void orc_update_many(const orc_config_t* cfg, int64_t u, int64_t j0, int64_t n,
                     const int32_t* rec_input, float* v, float* ca, uint8_t* ref, uint8_t* spk,
                     float* na);

/* Brute-force recurrent input (2^-16 mV) arriving at step t_arr at each of nt target
 * neurons, from the spikes emitted at steps e <= t_emit_max: mask[e - mask_t0][i] != 0 iff
 * neuron i spiked at step e, for e in [mask_t0, mask_t0 + mask_steps) (no spikes outside). */
void orc_input_brute(const orc_config_t* cfg, int64_t nt, const int64_t* targets, int64_t t_arr,
                     int64_t t_emit_max, const uint8_t* mask, int64_t mask_t0, int64_t mask_steps,
                     int32_t* out);

/* Initial membrane potential of neuron j; orc_initial_state also gives the second state
 * variable (Ca = 0 for LIF, the recovery variable u = b v for Izhikevich). */
float orc_initial_v(const orc_config_t* cfg, int64_t j);
void orc_initial_state(const orc_config_t* cfg, int64_t j, float* v, float* ca);

/* ---- simulation -------------------------------------------------------- */
typedef struct orc_sim orc_sim_t;

/* The CSR is borrowed (caller keeps it alive); w32 holds 2^-16 mV integer efficacies. */
orc_sim_t* orc_sim_create(const orc_config_t* cfg, int64_t n, const int64_t* row_ptr,
                          const int32_t* tgt, const uint8_t* dly, const int32_t* w32);
void orc_sim_destroy(orc_sim_t* s);
/* Advance n_steps steps (trajectory kept while recording is on, see orc_sim_record). */
int orc_sim_step(orc_sim_t* s, int64_t n_steps);
int64_t orc_sim_now(const orc_sim_t* s);
int32_t orc_sim_ring_slots(const orc_sim_t* s);

/* Spikes of step u (ascending ids); returns count, or -(count) if cap is short. */
int64_t orc_sim_spikes(const orc_sim_t* s, int64_t u, int32_t* ids, int64_t cap);
/* Totals: spikes, recurrent events (counted at emission), external events. */
void orc_sim_counts(const orc_sim_t* s, int64_t* spikes, int64_t* e_rec, int64_t* e_ext);
/* Sum of every input value taken out of the ring so far (2^-16 mV, as int64). */
int64_t orc_sim_consumed(const orc_sim_t* s);

/* State: V, Ca, ref (n each) and the pending input ring pend[D][n], where pend[q][j] is the
 * input already delivered to neuron j for step now+q.  With plasticity on, pend[q][j] is what
 * the spikes already emitted will bring with the weights they have now (plus any input set
 * or injected); orc_sim_set_state forgets the spikes before `now` and keeps the weights and
 * traces. */
void orc_sim_get_state(const orc_sim_t* s, float* v, float* ca, uint8_t* ref, int32_t* pend);
void orc_sim_set_state(orc_sim_t* s, int64_t now, const float* v, const float* ca,
                       const uint8_t* ref, const int32_t* pend);
/* The sodium-dependent AHP variable of every neuron (n). */
void orc_sim_get_na(const orc_sim_t* s, float* na);
void orc_sim_set_na(orc_sim_t* s, const float* na);
/* Test hook: add value (2^-16 mV) to the input of neuron j at step now+q. */
void orc_sim_inject(orc_sim_t* s, int32_t q, int64_t j, int32_t value);

/* Synaptic weights (2^-14 mV) of every synapse in CSR order: the generated ones, changed by
 * plasticity when it is on. */
void orc_sim_get_weights(const orc_sim_t* s, int16_t* wq);

/* The plasticity rule of orc_sim_step on one synapse of delay d, given its source's and its
 * target's spike flags pre[u], post[u] for steps u in [0, T) and its weight q0 at step 0:
 * the weight after step T - 1 (the same float32 traces and order as the simulation). */
int16_t orc_stdp_synapse(const orc_config_t* cfg, int64_t T, const uint8_t* pre,
                         const uint8_t* post, int32_t d, int16_t q0);

/* Trajectory recording: when enabled, every later step stores, per neuron, V before the
 * step, Ca before the step, the pre-threshold potential (0 when refractory), the spike
 * flag, the refractory flag and the consumed int32 input A. */
void orc_sim_record(orc_sim_t* s, int on);
/* Copy recorded steps [0, n_rec) out; arrays are [n_rec][n]. Returns n_rec. */
int64_t orc_sim_trajectory(const orc_sim_t* s, float* v_prev, float* ca_prev, float* v_tilde,
                           uint8_t* spk, uint8_t* refr, int32_t* input, int64_t cap_steps);

/* ---- adjoint (dpsnn_adjoint.c) ---------------------------------------------- */
typedef struct {
  double pm, pc, gamma, alpha, theta, vreset; /* step constants as used by the forward */
  double beta;                                /* surrogate slope, 1/mV */
} orc_adj_params_t;

/* Reverse recursion over a recorded trajectory ([T][n] arrays; s may be soft, r = refractory
 * flags).  w in mV per synapse of the CSR.  dl_ds: direct dL/ds, [T][n]; dl_dvt (nullable):
 * direct dL/dV~, [T][n].  Outputs: dL/dw per synapse, dL/dP_m, dL/dgamma.  Returns 0, or -1
 * if out of memory. */
int orc_adjoint(const orc_adj_params_t* k, int64_t n, int64_t T, const int64_t* row_ptr,
                const int32_t* tgt, const uint8_t* dly, const double* w, const double* v_prev,
                const double* ca_prev, const double* v_tilde, const double* s, const uint8_t* r,
                const double* dl_ds, const double* dl_dvt, double* grad_w, double* grad_pm,
                double* grad_gamma);

/* Smooth version of the step in FP64 (soft spike, soft reset and delivery, no refractory
 * period); records the trajectory ([T][n] outputs). */
int orc_soft_forward(const orc_config_t* cfg, const orc_adj_params_t* k, int64_t n, int64_t T,
                     const int64_t* row_ptr, const int32_t* tgt, const uint8_t* dly,
                     const double* w, double* v_prev, double* ca_prev, double* v_tilde,
                     double* s);

#ifdef __cplusplus
}
#endif
#endif
