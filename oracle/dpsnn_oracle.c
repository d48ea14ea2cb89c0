/*
 * dpsnn_oracle.c -- plain, slow CPU oracle of the DPSNN per-1 ms simulation step.
 *
 * TEST INFRASTRUCTURE ONLY (see dpsnn_oracle.h).  Written for readability, not speed:
 * every neuron and every synapse is visited with ordinary loops, in the order the
 * method describes.  Build with -O2 -ffp-contract=off so that float32 expressions are
 * evaluated exactly as written.
 */
#include "dpsnn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Threads.  Loops over independent rows or neurons may run on several host threads
 * (OpenMP); every result is the same for any thread count, because each row or neuron is
 * computed on its own and the synaptic input is an integer sum (order independent).
 * ------------------------------------------------------------------------- */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int32_t orc_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64
 * multiplications with the constants below, the high halves xor-ed with the other
 * two counter words and the key, the key bumped by the Weyl constants between rounds.
 * ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)prod1;
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)prod0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const orc_config_t* cfg, uint32_t a, uint32_t b, uint32_t c, uint32_t stream,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {a, b, c, stream};
  uint32_t key[2] = {(uint32_t)(cfg->seed & 0xffffffffu), (uint32_t)(cfg->seed >> 32)};
  orc_philox(ctr, key, out);
}

/* ---------------------------------------------------------------------------
 * Network (paper section 2, Methods).  Columns sit on a rows x cols grid, periodic in
 * both directions.  Column c = y*cols + x, neuron j = c*npc + k, k < n_exc excitatory
 * (80 % / 20 % split).  A neuron projects to its own column with pair probability p_own
 * and to the columns of a stencil around it with a probability that falls with the
 * distance r between column centres:
 *  - the 3x3 kernel: a total share p_remote of the row over the 8 surrounding columns,
 *    each weighted by exp(-r/decay) (r = 1 or sqrt 2 spacings);
 *  - the Gaussian kernel (the paper's lateral connectivity): lateral_amp exp(-r^2/2sigma^2)
 *    for every offset whose exp(-r^2/2sigma^2) reaches the cut-off (1/1000 in the paper,
 *    which leaves the 7x7 square minus its corners when sigma is the column spacing).
 * When the grid is so small that several stencil offsets land on the same column, the
 * offsets' probabilities are added, in stencil order (dy outer, dx inner, both ascending).
 * ------------------------------------------------------------------------- */
static double gauss_factor(const orc_config_t* cfg, int dy, int dx) {
  double r2 = (double)(dy * dy + dx * dx) * cfg->spacing_um * cfg->spacing_um;
  return exp(-r2 / (2.0 * cfg->lateral_sigma_um * cfg->lateral_sigma_um));
}

int32_t orc_stencil_radius(const orc_config_t* cfg) {
  if (cfg->conn_kernel != ORC_CONN_GAUSS) return 1;
  int32_t r = 0;
  while (r < 3 && gauss_factor(cfg, 0, r + 1) >= cfg->lateral_cutoff) ++r;
  return r;
}

static double offset_probability(const orc_config_t* cfg, int dy, int dx) {
  if (dy == 0 && dx == 0) return cfg->p_own;
  if (cfg->conn_kernel == ORC_CONN_GAUSS) {
    double g = gauss_factor(cfg, dy, dx);
    return g >= cfg->lateral_cutoff ? cfg->lateral_amp * g : 0.0;
  }
  double edge = exp(-(cfg->spacing_um / cfg->decay_um));
  double diag = exp(-(sqrt(2.0) * cfg->spacing_um / cfg->decay_um));
  double norm = 4.0 * edge + 4.0 * diag;
  double one = (dy == 0 || dx == 0) ? edge : diag;
  return cfg->p_remote * one / norm;
}

double orc_column_probability(const orc_config_t* cfg, int32_t src_col, int32_t tgt_col) {
  int sy = src_col / cfg->cols, sx = src_col % cfg->cols;
  int R = orc_stencil_radius(cfg);
  double p = 0.0;
  for (int dy = -R; dy <= R; ++dy) {
    for (int dx = -R; dx <= R; ++dx) {
      int ty = ((sy + dy) % cfg->rows + cfg->rows) % cfg->rows;
      int tx = ((sx + dx) % cfg->cols + cfg->cols) % cfg->cols;
      if (ty * cfg->cols + tx == tgt_col) p = p + offset_probability(cfg, dy, dx);
    }
  }
  return p;
}

/* Integer threshold of a probability: connect iff the 32-bit uniform is below it. */
static uint64_t prob_threshold(double p) {
  double t = floor(p * 4294967296.0);
  if (t <= 0.0) return 0;
  if (t >= 4294967296.0) return (uint64_t)1 << 32;
  return (uint64_t)t;
}

/* One pair: a Bernoulli trial with the column-pair probability, then an integer delay
 * uniform on [d_min, d_max] and a normal weight (sum of twelve 16-bit uniforms, the
 * Irwin-Hall approximation, bounded at 6 sigma) quantised to 2^-14 mV. */
static int pair_given_threshold(const orc_config_t* cfg, int64_t i, int64_t j, uint64_t thr,
                                int32_t* delay, int16_t* wq) {
  if (i == j) return 0;
  uint32_t r[4], r2[4];
  draw(cfg, (uint32_t)j, (uint32_t)i, 0u, ORC_STREAM_SYN, r);
  if ((uint64_t)r[0] >= thr) return 0;
  uint32_t span = (uint32_t)(cfg->d_max - cfg->d_min + 1);
  *delay = cfg->d_min + (int32_t)(((uint64_t)r[1] * (uint64_t)span) >> 32);
  draw(cfg, (uint32_t)j, (uint32_t)i, 1u, ORC_STREAM_SYN, r2);
  uint32_t words[6] = {r[2], r[3], r2[0], r2[1], r2[2], r2[3]};
  int32_t sum = 0;
  for (int q = 0; q < 6; ++q) sum += (int32_t)(words[q] & 0xffffu) + (int32_t)(words[q] >> 16);
  double z = (double)(sum - 393210) / 65536.0;
  int exc = (int32_t)(i % cfg->npc) < cfg->n_exc;
  double mu = exc ? cfg->we_mu : cfg->wi_mu;
  double sigma = exc ? cfg->we_sigma : cfg->wi_sigma;
  double w = mu + sigma * z;
  *wq = (int16_t)rint(w * 16384.0);
  return 1;
}

int orc_pair(const orc_config_t* cfg, int64_t i, int64_t j, int32_t* delay, int16_t* wq) {
  int32_t ci = (int32_t)(i / cfg->npc), cj = (int32_t)(j / cfg->npc);
  uint64_t thr = prob_threshold(orc_column_probability(cfg, ci, cj));
  return pair_given_threshold(cfg, i, j, thr, delay, wq);
}

typedef struct { int32_t d, j; int16_t w; } syn_t;

static int syn_order(const void* a, const void* b) {
  const syn_t* x = (const syn_t*)a;
  const syn_t* y = (const syn_t*)b;
  if (x->d != y->d) return x->d < y->d ? -1 : 1;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  return 0;
}

/* The distinct columns of the stencil of column c (each once, in stencil order); returns
 * how many. */
static int stencil_columns(const orc_config_t* cfg, int32_t c, int32_t out[49]) {
  int R = orc_stencil_radius(cfg);
  int y = c / cfg->cols, x = c % cfg->cols, n = 0;
  for (int dy = -R; dy <= R; ++dy) {
    for (int dx = -R; dx <= R; ++dx) {
      if (offset_probability(cfg, dy, dx) <= 0.0 && !(dy == 0 && dx == 0)) continue;
      int ty = ((y + dy) % cfg->rows + cfg->rows) % cfg->rows;
      int tx = ((x + dx) % cfg->cols + cfg->cols) % cfg->cols;
      int32_t t = ty * cfg->cols + tx, dup = 0;
      for (int q = 0; q < n; ++q) dup |= out[q] == t;
      if (!dup) out[n++] = t;
    }
  }
  return n;
}

int64_t orc_row(const orc_config_t* cfg, int64_t i, int32_t* tgt, uint8_t* dly, int16_t* wq,
                int64_t cap) {
  int32_t ci = (int32_t)(i / cfg->npc);
  int32_t cols[49];
  int ncand = stencil_columns(cfg, ci, cols);
  syn_t* tmp = (syn_t*)malloc(sizeof(syn_t) * (size_t)(ncand * cfg->npc + 1));
  int64_t n = 0;
  for (int q = 0; q < ncand; ++q) {
    int32_t c = cols[q];
    double p = orc_column_probability(cfg, ci, c);
    if (p <= 0.0) continue;
    uint64_t thr = prob_threshold(p);
    for (int32_t k = 0; k < cfg->npc; ++k) {
      int64_t j = (int64_t)c * cfg->npc + k;
      int32_t d; int16_t w;
      if (pair_given_threshold(cfg, i, j, thr, &d, &w)) { tmp[n].d = d; tmp[n].j = (int32_t)j; tmp[n].w = w; ++n; }
    }
  }
  qsort(tmp, (size_t)n, sizeof(syn_t), syn_order);
  if (n > cap) { free(tmp); return -1; }
  for (int64_t q = 0; q < n; ++q) { tgt[q] = tmp[q].j; dly[q] = (uint8_t)tmp[q].d; wq[q] = tmp[q].w; }
  free(tmp);
  return n;
}

/* The whole network: every row by orc_row.  Rows are independent, so blocks of rows are
 * built in parallel, each into a buffer of its own, and then laid out in row order. */
int64_t orc_network(const orc_config_t* cfg, int64_t* row_ptr, int32_t* tgt, uint8_t* dly,
                    int16_t* wq, int64_t cap) {
  const int64_t n = (int64_t)cfg->rows * cfg->cols * cfg->npc;
  const int64_t B = 256;                 /* rows per block */
  const int64_t nb = (n + B - 1) / B;
  const int64_t row_cap = 49 * (int64_t)cfg->npc;
  int32_t** btgt = (int32_t**)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int32_t*));
  uint8_t** bdly = (uint8_t**)calloc((size_t)(nb > 0 ? nb : 1), sizeof(uint8_t*));
  int16_t** bwq = (int16_t**)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int16_t*));
  int failed = 0;
  row_ptr[0] = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t i0 = b * B, i1 = i0 + B < n ? i0 + B : n;
    const int64_t bcap = (i1 - i0) * row_cap;
    int32_t* t = (int32_t*)malloc(sizeof(int32_t) * (size_t)bcap);
    uint8_t* d = (uint8_t*)malloc((size_t)bcap);
    int16_t* w = (int16_t*)malloc(sizeof(int16_t) * (size_t)bcap);
    int64_t used = 0;
    for (int64_t i = i0; i < i1 && t && d && w; ++i) {
      const int64_t len = orc_row(cfg, i, t + used, d + used, w + used, bcap - used);
      if (len < 0) break;
      row_ptr[i + 1] = len;  /* the row's length for now; turned into offsets below */
      used += len;
    }
    btgt[b] = t;
    bdly[b] = d;
    bwq[b] = w;
    if (!t || !d || !w) {
#pragma omp atomic write
      failed = 1;
    }
  }
  for (int64_t i = 0; i < n && !failed; ++i) row_ptr[i + 1] += row_ptr[i];
  if (!failed && row_ptr[n] > cap) failed = 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nb; ++b) {
    if (!failed) {
      const int64_t i0 = b * B, i1 = i0 + B < n ? i0 + B : n;
      const int64_t o = row_ptr[i0], len = row_ptr[i1] - row_ptr[i0];
      memcpy(tgt + o, btgt[b], sizeof(int32_t) * (size_t)len);
      memcpy(dly + o, bdly[b], (size_t)len);
      memcpy(wq + o, bwq[b], sizeof(int16_t) * (size_t)len);
    }
    free(btgt[b]);
    free(bdly[b]);
    free(bwq[b]);
  }
  free(btgt);
  free(bdly);
  free(bwq);
  return failed ? -1 : row_ptr[n];
}

/* ---------------------------------------------------------------------------
 * External input (paper section 2: external synapses as extra excitatory input).  Each
 * neuron has ext_syn independent Poisson synapses of rate ext_rate_hz, so the number of
 * external events arriving in one step is Poisson with mean ext_syn * rate * dt.  The
 * count is drawn by inverse CDF against integer thresholds, capped at 63.
 * ------------------------------------------------------------------------- */
void orc_poisson_table(double lam, uint64_t tab[63]) {
  double pk = exp(-lam);
  double cdf = 0.0;
  for (int k = 0; k < 63; ++k) {
    if (k > 0) pk = pk * lam / (double)k;
    cdf = cdf + pk;
    double t = floor(cdf * 4294967296.0);
    tab[k] = t >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)t;
  }
}

int32_t orc_poisson_count(const uint64_t tab[63], uint32_t x) {
  int32_t n = 0;
  for (int k = 0; k < 63; ++k)
    if (tab[k] <= (uint64_t)x) n += 1;
  return n;
}

/* The 32-bit uniform of neuron j at step u: one Philox block serves four consecutive
 * neurons, neuron j taking word j mod 4 of the block at counter (j / 4, u, 0, EXT). */
static uint32_t ext_uniform(const orc_config_t* cfg, int64_t j, int64_t u) {
  uint32_t r[4];
  draw(cfg, (uint32_t)(j >> 2), (uint32_t)u, 0u, ORC_STREAM_EXT, r);
  return r[j & 3];
}

void orc_ext_counts(const orc_config_t* cfg, int64_t u, int64_t j0, int64_t n, int32_t* out) {
  uint64_t tab[63];
  orc_poisson_table((double)cfg->ext_syn * cfg->ext_rate_hz * cfg->dt * 1e-3, tab);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n; ++q) out[q] = orc_poisson_count(tab, ext_uniform(cfg, j0 + q, u));
}

/* Initial state.  LIF: potential uniform on [0, v_reset) (24 random bits scaled exactly,
 * times v_reset), no calcium.  Izhikevich: potential uniform on [c, c + 5) mV around the
 * reset value and recovery u = b v (the resting relation), in float32. */
static int is_excitatory(const orc_config_t* cfg, int64_t j) {
  return (int32_t)(j % cfg->npc) < cfg->n_exc;
}

void orc_initial_state(const orc_config_t* cfg, int64_t j, float* v, float* ca) {
  uint32_t r[4];
  draw(cfg, (uint32_t)j, 0u, 0u, ORC_STREAM_INIT, r);
  float unit = (float)(r[0] >> 8) * 0x1p-24f;
  if (cfg->neuron_model == ORC_NEURON_IZHIKEVICH) {
    int e = is_excitatory(cfg, j);
    float c = (float)(e ? cfg->izh_c_e : cfg->izh_c_i);
    float b = (float)(e ? cfg->izh_b_e : cfg->izh_b_i);
    float spread = 5.0f * unit;
    *v = c + spread;
    *ca = b * *v;
  } else {
    *v = (float)cfg->v_reset * unit;
    *ca = 0.0f;
  }
}

float orc_initial_v(const orc_config_t* cfg, int64_t j) {
  float v, ca;
  orc_initial_state(cfg, j, &v, &ca);
  return v;
}

/* ---------------------------------------------------------------------------
 * Simulation state and the step (paper section 1: time-driven neuron update,
 * event-driven synaptic delivery; section 2: LIF neurons with calcium-driven
 * after-hyperpolarisation).
 * ------------------------------------------------------------------------- */
struct orc_sim {
  orc_config_t cfg;
  int64_t n;
  const int64_t* row_ptr;
  const int32_t* tgt;
  const uint8_t* dly;
  const int32_t* w32;
  int32_t D;            /* ring slots: d_max + 1 */
  uint64_t ptab[63];
  float* v;
  float* ca;            /* calcium (LIF) or recovery variable u (Izhikevich) */
  float* na;            /* sodium-dependent AHP variable (LIF) */
  uint8_t* ref;
  uint32_t* ring;       /* [D][n]; slot u % D holds the input of step u */
  int64_t now;
  uint8_t* spiked;      /* [n] spike flags of the step being computed */
  /* plasticity (cfg.stdp): current weights, traces and the synapses into each neuron */
  int16_t* q;           /* [S] weights, 2^-14 mV */
  float* xr;            /* [D][n] presynaptic trace of steps u - D + 1 .. u, slot u % D */
  float* y;             /* [n] postsynaptic trace after the last step */
  float* ym;            /* [n] postsynaptic trace decayed to the current step */
  int32_t* in_now;      /* [n] input of the current step */
  int64_t* in_ptr;      /* [n+1] incoming synapses of each neuron ... */
  int64_t* in_syn;      /* ... their CSR indices */
  int32_t* src_of;      /* [S] source neuron of each synapse */
  /* raster: spike ids of all steps, with per-step offsets */
  int32_t* sp_ids; int64_t sp_n, sp_cap;
  int64_t* sp_off; int64_t off_cap;
  int64_t e_rec, e_ext;
  int64_t consumed;     /* sum of all inputs taken out of the ring (checksum) */
  /* trajectory recording */
  int rec_on; int64_t rec_n, rec_cap;
  float *r_vprev, *r_caprev, *r_vt; uint8_t *r_s, *r_r; int32_t* r_in;
};

orc_sim_t* orc_sim_create(const orc_config_t* cfg, int64_t n, const int64_t* row_ptr,
                          const int32_t* tgt, const uint8_t* dly, const int32_t* w32) {
  orc_sim_t* s = (orc_sim_t*)calloc(1, sizeof(orc_sim_t));
  s->cfg = *cfg;
  s->n = n;
  s->row_ptr = row_ptr; s->tgt = tgt; s->dly = dly; s->w32 = w32;
  s->D = cfg->d_max + 1;
  orc_poisson_table((double)cfg->ext_syn * cfg->ext_rate_hz * cfg->dt * 1e-3, s->ptab);
  s->v = (float*)malloc(sizeof(float) * (size_t)n);
  s->ca = (float*)calloc((size_t)n, sizeof(float));
  s->na = (float*)calloc((size_t)(n > 0 ? n : 1), sizeof(float));
  s->ref = (uint8_t*)calloc((size_t)n, 1);
  s->ring = (uint32_t*)calloc((size_t)s->D * (size_t)n, sizeof(uint32_t));
  s->spiked = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  for (int64_t j = 0; j < n; ++j) orc_initial_state(cfg, j, &s->v[j], &s->ca[j]);
  if (cfg->stdp) {
    int64_t S = row_ptr[n];
    s->q = (int16_t*)malloc(sizeof(int16_t) * (size_t)(S > 0 ? S : 1));
    for (int64_t e = 0; e < S; ++e) s->q[e] = (int16_t)(w32[e] / 4);
    s->xr = (float*)calloc((size_t)s->D * (size_t)n, sizeof(float));
    s->y = (float*)calloc((size_t)n, sizeof(float));
    s->ym = (float*)calloc((size_t)n, sizeof(float));
    s->in_now = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    /* the synapses into each neuron: a counting sort of the CSR by target */
    s->in_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    s->in_syn = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
    s->src_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S > 0 ? S : 1));
    for (int64_t e = 0; e < S; ++e) s->in_ptr[tgt[e] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) s->in_ptr[j + 1] += s->in_ptr[j];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) fill[j] = s->in_ptr[j];
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        s->src_of[e] = (int32_t)i;
        s->in_syn[fill[tgt[e]]++] = e;
      }
    free(fill);
  }
  s->off_cap = 1024;
  s->sp_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)s->off_cap);
  s->sp_off[0] = 0;
  s->sp_cap = 1024;
  s->sp_ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)s->sp_cap);
  return s;
}

void orc_sim_destroy(orc_sim_t* s) {
  if (!s) return;
  free(s->v); free(s->ca); free(s->na); free(s->ref); free(s->ring); free(s->spiked);
  free(s->q); free(s->xr); free(s->y); free(s->ym); free(s->in_now); free(s->in_ptr);
  free(s->in_syn); free(s->src_of);
  free(s->sp_ids); free(s->sp_off);
  free(s->r_vprev); free(s->r_caprev); free(s->r_vt); free(s->r_s); free(s->r_r);
  free(s->r_in);
  free(s);
}

void orc_sim_record(orc_sim_t* s, int on) { s->rec_on = on; }

static void push_spike(orc_sim_t* s, int32_t j) {
  if (s->sp_n == s->sp_cap) {
    s->sp_cap *= 2;
    s->sp_ids = (int32_t*)realloc(s->sp_ids, sizeof(int32_t) * (size_t)s->sp_cap);
  }
  s->sp_ids[s->sp_n++] = j;
}

static void grow_record(orc_sim_t* s) {
  if (s->rec_n < s->rec_cap) return;
  s->rec_cap = s->rec_cap ? 2 * s->rec_cap : 64;
  size_t m = (size_t)s->rec_cap * (size_t)s->n;
  s->r_vprev = (float*)realloc(s->r_vprev, sizeof(float) * m);
  s->r_caprev = (float*)realloc(s->r_caprev, sizeof(float) * m);
  s->r_vt = (float*)realloc(s->r_vt, sizeof(float) * m);
  s->r_s = (uint8_t*)realloc(s->r_s, m);
  s->r_r = (uint8_t*)realloc(s->r_r, m);
  s->r_in = (int32_t*)realloc(s->r_in, sizeof(int32_t) * m);
}

/* Neuron constants, computed in double and rounded once to float. */
typedef struct {
  int32_t model;
  float pm, pc, gam, alpha, theta, vreset;
  float pna, gna, alpha_na;        /* sodium-dependent AHP */
  float ia[2], ib[2], ic[2], id[2], vpeak;  /* Izhikevich: [0] excitatory, [1] inhibitory */
  int32_t jfx, tref;
} consts_t;

static consts_t constants_of(const orc_config_t* cfg) {
  consts_t k;
  k.model = cfg->neuron_model;
  k.pm = (float)exp(-cfg->dt / cfg->tau_m);
  k.pc = (float)exp(-cfg->dt / cfg->tau_ca);
  k.gam = (float)(cfg->g_ahp * cfg->dt);
  k.alpha = (float)cfg->ca_inc;
  k.theta = (float)cfg->theta;
  k.vreset = (float)cfg->v_reset;
  k.pna = cfg->tau_na > 0.0 ? (float)exp(-cfg->dt / cfg->tau_na) : 0.0f;
  k.gna = (float)(cfg->g_na * cfg->dt);
  k.alpha_na = (float)cfg->na_inc;
  k.ia[0] = (float)cfg->izh_a_e; k.ib[0] = (float)cfg->izh_b_e;
  k.ic[0] = (float)cfg->izh_c_e; k.id[0] = (float)cfg->izh_d_e;
  k.ia[1] = (float)cfg->izh_a_i; k.ib[1] = (float)cfg->izh_b_i;
  k.ic[1] = (float)cfg->izh_c_i; k.id[1] = (float)cfg->izh_d_i;
  k.vpeak = (float)cfg->izh_vpeak;
  k.jfx = (int32_t)rint(cfg->j_ext * 65536.0);
  k.tref = cfg->neuron_model == ORC_NEURON_IZHIKEVICH ? 0 : cfg->t_ref;
  return k;
}

/* Half a millisecond of the Izhikevich membrane equation (Izhikevich, "Simple model of
 * spiking neurons", IEEE TNN 2003): v' = 0.04 v^2 + 5 v + 140 - u + I, one Euler step of
 * 0.5 ms, the terms added from left to right. */
static float izh_half_step(float v, float u, float cur) {
  float sq = v * v;
  float quad = 0.04f * sq;
  float lin = 5.0f * v;
  float rhs = quad + lin;
  rhs = rhs + 140.0f;
  rhs = rhs - u;
  rhs = rhs + cur;
  float half = 0.5f * rhs;
  return v + half;
}

/* The neuron part of a step.  The input is A = recurrent input + n_ext * J_ext (int32,
 * wrap-around), I = A 2^-16 mV.
 * LIF with spike-frequency adaptation (paper section 2: calcium- and sodium-dependent AHP
 * currents):
 *  - a refractory neuron counts down, stays at V_reset and discards its input;
 *  - otherwise V~ = (((P_m V) - (gamma Ca)) - (gamma_Na Na)) + I, with P_m = exp(-dt/tau_m),
 *    gamma = g_AHP dt and gamma_Na = g_Na dt; a spike is emitted if V~ >= theta, then
 *    V <- V_reset and the refractory counter is set;
 *  - Ca <- P_c Ca + alpha s and Na <- P_Na Na + alpha_Na s, P_x = exp(-dt/tau_x).
 *  With g_Na = 0 the sodium term is an exact zero and the step is the one-variable model.
 * Izhikevich neurons (the earlier report's RS/FS neurons; Izhikevich, IEEE TNN 2003): two
 * half-millisecond Euler steps of v' = 0.04 v^2 + 5 v + 140 - u + I, then
 * u <- u + a (b v - u) with the new v; a spike if v >= v_peak, then v <- c and u <- u + d
 * (a, b, c, d of the neuron's type: RS for excitatory, FS for inhibitory neurons); no
 * refractory period.  The recovery variable u lives where LIF keeps Ca.
 * Returns the spike flag; *vt receives V~ (the potential before the reset; 0 when
 * refractory), *refr the refractory flag, *a_out the consumed input. */
static int neuron_update(const consts_t* k, int excit, uint32_t rec_input, int32_t n_ext, float* v,
                         float* ca, float* na, uint8_t* ref, float* vt_out, int* refr_out,
                         uint32_t* a_out) {
  uint32_t a = rec_input + (uint32_t)n_ext * (uint32_t)k->jfx;
  float cur = (float)(int32_t)a * 0x1p-16f;
  float vprev = *v, caprev = *ca;
  float vt = 0.0f;
  int spike = 0, refr = 0;
  if (k->model == ORC_NEURON_IZHIKEVICH) {
    int t = excit ? 0 : 1;
    float v1 = izh_half_step(vprev, caprev, cur);
    float v2 = izh_half_step(v1, caprev, cur);
    float bv = k->ib[t] * v2;
    float gap = bv - caprev;
    float du = k->ia[t] * gap;
    float unew = caprev + du;
    vt = v2;
    if (v2 >= k->vpeak) {
      spike = 1;
      *v = k->ic[t];
      *ca = unew + k->id[t];
    } else {
      *v = v2;
      *ca = unew;
    }
    *vt_out = vt; *refr_out = 0; *a_out = a;
    return spike;
  }
  float naprev = na ? *na : 0.0f;
  if (*ref > 0) {
    refr = 1;
    *ref -= 1;
    *v = k->vreset;
  } else {
    float leak = k->pm * vprev;
    float ahp = k->gam * caprev;
    float drop = leak - ahp;
    float ahp_na = k->gna * naprev;
    drop = drop - ahp_na;
    vt = drop + cur;
    if (vt >= k->theta) {
      spike = 1;
      *v = k->vreset;
      *ref = (uint8_t)k->tref;
    } else {
      *v = vt;
    }
  }
  float decayed = k->pc * caprev;
  *ca = decayed + (spike ? k->alpha : 0.0f);
  if (na) {
    float na_decayed = k->pna * naprev;
    *na = na_decayed + (spike ? k->alpha_na : 0.0f);
  }
  *vt_out = vt; *refr_out = refr; *a_out = a;
  return spike;
}

int orc_neuron_update(const orc_config_t* cfg, int64_t j, int64_t u, int32_t rec_input, float* v,
                      float* ca, uint8_t* ref, float* na) {
  consts_t k = constants_of(cfg);
  int32_t n_ext;
  orc_ext_counts(cfg, u, j, 1, &n_ext);
  float vt; int refr; uint32_t a;
  return neuron_update(&k, is_excitatory(cfg, j), (uint32_t)rec_input, n_ext, v, ca, na, ref, &vt,
                       &refr, &a);
}

void orc_update_many(const orc_config_t* cfg, int64_t u, int64_t j0, int64_t n,
                     const int32_t* rec_input, float* v, float* ca, uint8_t* ref, uint8_t* spk,
                     float* na) {
  consts_t k = constants_of(cfg);
  int32_t* n_ext = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  orc_ext_counts(cfg, u, j0, n, n_ext);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n; ++q) {
    float vt; int refr; uint32_t a;
    spk[q] = (uint8_t)neuron_update(&k, is_excitatory(cfg, j0 + q), (uint32_t)rec_input[q],
                                    n_ext[q], &v[q], &ca[q], na ? &na[q] : NULL, &ref[q], &vt,
                                    &refr, &a);
  }
  free(n_ext);
}

/* Recurrent input by its definition, without a ring: the sum of the efficacies 4 w_q of
 * every synapse i -> j of delay d whose source spiked at step e = t_arr - d, over the
 * emission steps e <= t_emit_max covered by the spike mask.  The candidate sources are
 * all neurons of the (unique) columns of the stencil around j's column (the stencil is
 * symmetric); each pair is decided again from the generator's definition. */
void orc_input_brute(const orc_config_t* cfg, int64_t nt, const int64_t* targets, int64_t t_arr,
                     int64_t t_emit_max, const uint8_t* mask, int64_t mask_t0, int64_t mask_steps,
                     int32_t* out) {
  const int64_t n = (int64_t)cfg->rows * cfg->cols * cfg->npc;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t j = targets[t];
    const int32_t cj = (int32_t)(j / cfg->npc);
    int32_t cols[49];
    const int nsrc = stencil_columns(cfg, cj, cols);
    uint32_t acc = 0;
    for (int q = 0; q < nsrc; ++q) {
      const int32_t c = cols[q];
      for (int32_t k = 0; k < cfg->npc; ++k) {
        const int64_t i = (int64_t)c * cfg->npc + k;
        int32_t d; int16_t w;
        if (!orc_pair(cfg, i, j, &d, &w)) continue;
        const int64_t e = t_arr - d;
        if (e > t_emit_max || e < mask_t0 || e >= mask_t0 + mask_steps) continue;
        if (mask[(size_t)(e - mask_t0) * (size_t)n + (size_t)i]) acc += (uint32_t)(4 * (int32_t)w);
      }
    }
    out[t] = (int32_t)acc;
  }
}

/* One step u = now (paper section 1: every neuron is updated every step; synaptic work
 * follows the spikes):
 *  1. each neuron takes its input ring[u % D][j] (the slot is cleared), adds its external
 *     Poisson count times J_ext and is updated as in neuron_update;
 *  2. the spikes of the step are recorded in ascending order and counted as events (each
 *     outgoing synapse of a spiking neuron is one recurrent event; each external arrival
 *     is one external event);
 *  3. every synapse i->j of delay d of a spiking neuron i adds its efficacy to
 *     ring[(u + d) % D][j].
 * Neurons (1) and spikes (3) are independent of each other, so both loops may run on
 * several threads; the additions into the ring are atomic and the spike list is collected
 * in ascending order afterwards.
 *
 * With plasticity on (spike-timing-dependent plasticity; paper sections 1-2 name it, the
 * rule is not given there): the all-to-all pair rule with exponential windows, in weight
 * units of 2^-14 mV, on the synapses of excitatory sources (weights >= 0; inhibitory
 * weights are negative and stay fixed), bounded to [0, w_max].  Spikes arrive at u = t + d
 * carrying the weight they find then, so the input is gathered at arrival from the spikes of
 * the last d_max steps instead of being pushed into the ring at emission.  Step u:
 *  1. y-(j) = P- y(j), the postsynaptic trace decayed to u (spikes before u);
 *     every synapse i -> j whose source spiked at u - d adds 4 w to j's input, then is
 *     depressed: w <- max(0, w - rint(A- y-(j) 2^14));
 *  2. the neurons are updated as above;
 *  3. y(j) = y-(j) + s_j(u); x_u(i) = P+ x_{u-1}(i) + s_i(u), the presynaptic trace;
 *  4. every synapse i -> j (delay d) into a neuron j that spiked at u is potentiated:
 *     w <- min(w_max, w + rint(A+ x_{u-d}(i) 2^14)), x_{u-d}(i) counting the source's spikes
 *     up to u - d, i.e. its arrivals up to u; a change that rounds to 0 is none (the bound
 *     acts on changes only).
 * So every (arrival, postsynaptic spike) pair changes w once: by A+ exp(-(t_post - t_arr) /
 * tau+) if the spike is not earlier than the arrival, by -A- exp(-(t_arr - t_post) /
 * tau-) if it is (before rounding and bounds); P+- = exp(-dt / tau+-), float32. */
static void stdp_step(orc_sim_t* s, const consts_t* k);

int orc_sim_step(orc_sim_t* s, int64_t n_steps) {
  consts_t k = constants_of(&s->cfg);
  if (s->cfg.stdp) {
    for (int64_t it = 0; it < n_steps; ++it) stdp_step(s, &k);
    return 0;
  }
  for (int64_t it = 0; it < n_steps; ++it) {
    int64_t u = s->now;
    int64_t slot = u % s->D;
    uint32_t* in = s->ring + slot * s->n;
    int64_t first = s->sp_n;
    int64_t consumed = 0, e_ext = 0, e_rec = 0;
    if (s->rec_on) grow_record(s);
#pragma omp parallel for schedule(static) reduction(+ : consumed, e_ext)
    for (int64_t j = 0; j < s->n; ++j) {
      int32_t next = orc_poisson_count(s->ptab, ext_uniform(&s->cfg, j, u));
      float vprev = s->v[j], caprev = s->ca[j], vt;
      int refr;
      uint32_t a;
      int spike = neuron_update(&k, is_excitatory(&s->cfg, j), in[j], next, &s->v[j], &s->ca[j],
                                &s->na[j], &s->ref[j], &vt, &refr, &a);
      in[j] = 0;
      consumed += (int64_t)(int32_t)a;
      s->spiked[j] = (uint8_t)spike;
      e_ext += next;
      if (s->rec_on) {
        size_t o = (size_t)s->rec_n * (size_t)s->n + (size_t)j;
        s->r_vprev[o] = vprev; s->r_caprev[o] = caprev; s->r_vt[o] = vt;
        s->r_s[o] = (uint8_t)spike; s->r_r[o] = (uint8_t)refr; s->r_in[o] = (int32_t)a;
      }
    }
    s->consumed += consumed;
    s->e_ext += e_ext;
    for (int64_t j = 0; j < s->n; ++j)
      if (s->spiked[j]) push_spike(s, (int32_t)j);
    if (s->rec_on) s->rec_n += 1;
    if (orc_threads() == 1) {
      for (int64_t q = first; q < s->sp_n; ++q) {
        int64_t i = s->sp_ids[q];
        e_rec += s->row_ptr[i + 1] - s->row_ptr[i];
        for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
          int64_t dst = ((u + s->dly[e]) % s->D) * s->n + s->tgt[e];
          s->ring[dst] += (uint32_t)s->w32[e];
        }
      }
    } else {
      /* the same loop over spikes on several threads, each addition atomic */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : e_rec)
      for (int64_t q = first; q < s->sp_n; ++q) {
        int64_t i = s->sp_ids[q];
        e_rec += s->row_ptr[i + 1] - s->row_ptr[i];
        for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
          int64_t dst = ((u + s->dly[e]) % s->D) * s->n + s->tgt[e];
#pragma omp atomic update
          s->ring[dst] += (uint32_t)s->w32[e];
        }
      }
    }
    s->e_rec += e_rec;
    s->now += 1;
    if (s->now >= s->off_cap) {
      s->off_cap *= 2;
      s->sp_off = (int64_t*)realloc(s->sp_off, sizeof(int64_t) * (size_t)s->off_cap);
    }
    s->sp_off[s->now] = s->sp_n;
  }
  return 0;
}

static void next_step_offsets(orc_sim_t* s) {
  s->now += 1;
  if (s->now >= s->off_cap) {
    s->off_cap *= 2;
    s->sp_off = (int64_t*)realloc(s->sp_off, sizeof(int64_t) * (size_t)s->off_cap);
  }
  s->sp_off[s->now] = s->sp_n;
}

static void stdp_step(orc_sim_t* s, const consts_t* k) {
  const orc_config_t* c = &s->cfg;
  const int64_t u = s->now, n = s->n;
  const float pplus = (float)exp(-c->dt / c->stdp_tau_plus);
  const float pminus = (float)exp(-c->dt / c->stdp_tau_minus);
  const float aplus = (float)c->stdp_a_plus, aminus = (float)c->stdp_a_minus;
  const int32_t qmax = (int32_t)rint(c->stdp_w_max * 16384.0);
  /* input held in the ring (set by orc_sim_set_state or orc_sim_inject) comes first */
  uint32_t* ring = s->ring + (u % s->D) * n;
  for (int64_t j = 0; j < n; ++j) {
    s->ym[j] = pminus * s->y[j];
    s->in_now[j] = (int32_t)ring[j];
    ring[j] = 0;
  }
  /* 1. arrivals of the spikes of steps u - d, delivered with the current weight, then
   *    depression of the excitatory ones */
  for (int32_t d = c->d_min; d <= c->d_max; ++d) {
    const int64_t t = u - d;
    if (t < 0) continue;
    for (int64_t q = s->sp_off[t]; q < s->sp_off[t + 1]; ++q) {
      const int64_t i = s->sp_ids[q];
      for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
        if (s->dly[e] != d) continue;
        const int32_t j = s->tgt[e];
        s->in_now[j] = (int32_t)((uint32_t)s->in_now[j] + 4u * (uint32_t)(int32_t)s->q[e]);
        if (s->q[e] >= 0) {
          const float t1 = aminus * s->ym[j];
          const int32_t dq = (int32_t)rintf(t1 * 16384.0f);
          const int32_t w = s->q[e] - dq;
          s->q[e] = (int16_t)(w < 0 ? 0 : w);
        }
      }
    }
  }
  /* 2. the neurons */
  if (s->rec_on) grow_record(s);
  for (int64_t j = 0; j < n; ++j) {
    const int32_t next = orc_poisson_count(s->ptab, ext_uniform(c, j, u));
    const float vprev = s->v[j], caprev = s->ca[j];
    float vt;
    int refr;
    uint32_t a;
    const int spike = neuron_update(k, is_excitatory(c, j), (uint32_t)s->in_now[j], next,
                                    &s->v[j], &s->ca[j], &s->na[j], &s->ref[j], &vt, &refr, &a);
    s->consumed += (int64_t)(int32_t)a;
    s->e_ext += next;
    s->spiked[j] = (uint8_t)spike;
    if (spike) push_spike(s, (int32_t)j);
    if (s->rec_on) {
      size_t o = (size_t)s->rec_n * (size_t)n + (size_t)j;
      s->r_vprev[o] = vprev; s->r_caprev[o] = caprev; s->r_vt[o] = vt;
      s->r_s[o] = (uint8_t)spike; s->r_r[o] = (uint8_t)refr; s->r_in[o] = (int32_t)a;
    }
  }
  if (s->rec_on) s->rec_n += 1;
  /* 3. traces */
  float* xu = s->xr + (u % s->D) * n;
  const float* xp = s->xr + ((u + s->D - 1) % s->D) * n;
  for (int64_t j = 0; j < n; ++j) {
    const float decayed = pplus * xp[j];
    xu[j] = decayed + (s->spiked[j] ? 1.0f : 0.0f);
    s->y[j] = s->ym[j] + (s->spiked[j] ? 1.0f : 0.0f);
  }
  /* 4. potentiation of the excitatory synapses into the neurons that spiked */
  for (int64_t j = 0; j < n; ++j) {
    if (!s->spiked[j]) continue;
    for (int64_t q = s->in_ptr[j]; q < s->in_ptr[j + 1]; ++q) {
      const int64_t e = s->in_syn[q];
      const int64_t t = u - s->dly[e];
      if (s->q[e] < 0 || t < 0) continue;
      const float x = s->xr[(t % s->D) * n + s->src_of[e]];
      const float t1 = aplus * x;
      const int32_t dq = (int32_t)rintf(t1 * 16384.0f);
      if (dq == 0) continue;  /* no change: a weight above w_max stays until one comes */
      const int32_t w = s->q[e] + dq;
      s->q[e] = (int16_t)(w > qmax ? qmax : w);
    }
  }
  /* recurrent events at emission, as without plasticity */
  for (int64_t q = s->sp_off[u]; q < s->sp_n; ++q) {
    const int64_t i = s->sp_ids[q];
    s->e_rec += s->row_ptr[i + 1] - s->row_ptr[i];
  }
  next_step_offsets(s);
}

int16_t orc_stdp_synapse(const orc_config_t* c, int64_t T, const uint8_t* pre,
                         const uint8_t* post, int32_t d, int16_t q0) {
  if (q0 < 0 || T <= 0) return q0;
  const float pplus = (float)exp(-c->dt / c->stdp_tau_plus);
  const float pminus = (float)exp(-c->dt / c->stdp_tau_minus);
  const float aplus = (float)c->stdp_a_plus, aminus = (float)c->stdp_a_minus;
  const int32_t qmax = (int32_t)rint(c->stdp_w_max * 16384.0);
  float* x = (float*)malloc(sizeof(float) * (size_t)T);
  float y = 0.0f, xprev = 0.0f;
  int32_t q = q0;
  for (int64_t u = 0; u < T; ++u) {
    const float ym = pminus * y;
    if (u >= d && pre[u - d]) {  /* an arrival: depression by the target's earlier spikes */
      const float t1 = aminus * ym;
      const int32_t w = q - (int32_t)rintf(t1 * 16384.0f);
      q = w < 0 ? 0 : w;
    }
    y = ym + (post[u] ? 1.0f : 0.0f);
    const float decayed = pplus * xprev;
    x[u] = decayed + (pre[u] ? 1.0f : 0.0f);
    xprev = x[u];
    if (post[u] && u >= d) {     /* a target spike: potentiation by the arrivals up to u */
      const float t1 = aplus * x[u - d];
      const int32_t dq = (int32_t)rintf(t1 * 16384.0f);
      if (dq != 0) q = q + dq > qmax ? qmax : q + dq;
    }
  }
  free(x);
  return (int16_t)q;
}

void orc_sim_get_weights(const orc_sim_t* s, int16_t* wq) {
  const int64_t S = s->row_ptr[s->n];
  for (int64_t e = 0; e < S; ++e) wq[e] = s->q ? s->q[e] : (int16_t)(s->w32[e] / 4);
}

int64_t orc_sim_now(const orc_sim_t* s) { return s->now; }
int32_t orc_sim_ring_slots(const orc_sim_t* s) { return s->D; }

int64_t orc_sim_spikes(const orc_sim_t* s, int64_t u, int32_t* ids, int64_t cap) {
  if (u < 0 || u >= s->now) return 0;
  int64_t a = s->sp_off[u], b = s->sp_off[u + 1];
  if (b - a > cap) return -(b - a);
  for (int64_t q = a; q < b; ++q) ids[q - a] = s->sp_ids[q];
  return b - a;
}

void orc_sim_counts(const orc_sim_t* s, int64_t* spikes, int64_t* e_rec, int64_t* e_ext) {
  *spikes = s->sp_n; *e_rec = s->e_rec; *e_ext = s->e_ext;
}

int64_t orc_sim_consumed(const orc_sim_t* s) { return s->consumed; }

void orc_sim_get_state(const orc_sim_t* s, float* v, float* ca, uint8_t* ref, int32_t* pend) {
  memcpy(v, s->v, sizeof(float) * (size_t)s->n);
  memcpy(ca, s->ca, sizeof(float) * (size_t)s->n);
  memcpy(ref, s->ref, (size_t)s->n);
  if (s->cfg.stdp) {
    /* the input held in the ring plus what the spikes already emitted will bring at step
     * now + q, with today's weights */
    for (int32_t q = 0; q < s->D; ++q) {
      int64_t slot = (s->now + q) % s->D;
      for (int64_t j = 0; j < s->n; ++j) pend[q * s->n + j] = (int32_t)s->ring[slot * s->n + j];
    }
    for (int64_t t = s->now - s->cfg.d_max; t < s->now; ++t) {
      if (t < 0) continue;
      for (int64_t q = s->sp_off[t]; q < s->sp_off[t + 1]; ++q) {
        const int64_t i = s->sp_ids[q];
        for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
          const int64_t due = t + s->dly[e];
          if (due < s->now) continue;
          int32_t* p = &pend[(due - s->now) * s->n + s->tgt[e]];
          *p = (int32_t)((uint32_t)*p + 4u * (uint32_t)(int32_t)s->q[e]);
        }
      }
    }
    return;
  }
  for (int32_t q = 0; q < s->D; ++q) {
    int64_t slot = (s->now + q) % s->D;
    for (int64_t j = 0; j < s->n; ++j) pend[q * s->n + j] = (int32_t)s->ring[slot * s->n + j];
  }
}

void orc_sim_set_state(orc_sim_t* s, int64_t now, const float* v, const float* ca,
                       const uint8_t* ref, const int32_t* pend) {
  /* the raster restarts at step `now`: earlier steps are reported empty */
  if (now + 1 > s->off_cap) {
    s->off_cap = now + 1024;
    s->sp_off = (int64_t*)realloc(s->sp_off, sizeof(int64_t) * (size_t)s->off_cap);
  }
  for (int64_t q = 0; q <= now; ++q) s->sp_off[q] = s->sp_n;
  s->now = now;
  memcpy(s->v, v, sizeof(float) * (size_t)s->n);
  memcpy(s->ca, ca, sizeof(float) * (size_t)s->n);
  memcpy(s->ref, ref, (size_t)s->n);
  for (int32_t q = 0; q < s->D; ++q) {
    int64_t slot = (now + q) % s->D;
    for (int64_t j = 0; j < s->n; ++j) s->ring[slot * s->n + j] = (uint32_t)pend[q * s->n + j];
  }
}

void orc_sim_get_na(const orc_sim_t* s, float* na) {
  memcpy(na, s->na, sizeof(float) * (size_t)s->n);
}

void orc_sim_set_na(orc_sim_t* s, const float* na) {
  memcpy(s->na, na, sizeof(float) * (size_t)s->n);
}

void orc_sim_inject(orc_sim_t* s, int32_t q, int64_t j, int32_t value) {
  int64_t slot = (s->now + q) % s->D;
  s->ring[slot * s->n + j] += (uint32_t)value;
}

int64_t orc_sim_trajectory(const orc_sim_t* s, float* v_prev, float* ca_prev, float* v_tilde,
                           uint8_t* spk, uint8_t* refr, int32_t* input, int64_t cap_steps) {
  int64_t m = s->rec_n < cap_steps ? s->rec_n : cap_steps;
  size_t cnt = (size_t)m * (size_t)s->n;
  if (m > 0) {
    memcpy(v_prev, s->r_vprev, sizeof(float) * cnt);
    memcpy(ca_prev, s->r_caprev, sizeof(float) * cnt);
    memcpy(v_tilde, s->r_vt, sizeof(float) * cnt);
    memcpy(spk, s->r_s, cnt);
    memcpy(refr, s->r_r, cnt);
    memcpy(input, s->r_in, sizeof(int32_t) * cnt);
  }
  return m;
}
