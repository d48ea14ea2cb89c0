/*
 * abi_client.c -- a plain C program that uses libdpsnn.so through include/dpsnn.h only
 * (built by the tests with gcc, no HIP headers).
 *
 *   abi_client errors
 *       bad configurations and NULL arguments are refused with the documented codes before
 *       any device work (runs without a GPU); prints "errors ok".
 *   abi_client run STEPS key=value ...
 *       one network of the given parameters (the sim_config_t fields of the column recipe,
 *       plus rows, cols, seed, ext_rate_hz): sim_query_sizes, sim_create, STEPS steps,
 *       then the raster of every step through sim_read_spikes, one line per step:
 *       "step <u> <count> <ids...>", then "spikes e_rec e_ext" counters.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dpsnn.h"

static int fail(const char* what, int rc, const sim_t* sim) {
  fprintf(stderr, "%s: rc %d: %s\n", what, rc, sim_last_error(sim));
  return 1;
}

static void recipe(sim_config_t* c, sim_net_t* net) {
  memset(c, 0, sizeof(*c));
  memset(net, 0, sizeof(*net));
  c->npc = 1240; c->n_exc = 992;
  c->p_own = 0.6; c->p_remote = 0.4; c->decay_um = 100.0; c->spacing_um = 100.0;
  c->d_min = 1; c->d_max = 20;
  c->we_mu = 0.2; c->we_sigma = 0.02; c->wi_mu = -0.8; c->wi_sigma = 0.08;
  c->tau_m = 20.0; c->theta = 20.0; c->v_reset = 15.0; c->t_ref = 2;
  c->tau_ca = 300.0; c->ca_inc = 0.05; c->g_ahp = 0.2; c->dt = 1.0;
  c->ext_syn = 1000; c->j_ext = 0.3;
  net->rows = 2; net->cols = 2; net->seed = 0; net->ext_rate_hz = 3.0;
  c->n_nets = 1;
  c->nets = net;
}

static int set_field(sim_config_t* c, sim_net_t* n, const char* kv) {
  char key[64];
  const char* eq = strchr(kv, '=');
  if (!eq || (size_t)(eq - kv) >= sizeof(key)) return -1;
  memcpy(key, kv, (size_t)(eq - kv));
  key[eq - kv] = 0;
  const char* v = eq + 1;
#define INT(f) if (!strcmp(key, #f)) { c->f = (int32_t)atol(v); return 0; }
#define DBL(f) if (!strcmp(key, #f)) { c->f = atof(v); return 0; }
  INT(npc) INT(n_exc) INT(d_min) INT(d_max) INT(t_ref) INT(ext_syn)
  DBL(p_own) DBL(p_remote) DBL(decay_um) DBL(spacing_um) DBL(we_mu) DBL(we_sigma)
  DBL(wi_mu) DBL(wi_sigma) DBL(tau_m) DBL(theta) DBL(v_reset) DBL(tau_ca) DBL(ca_inc)
  DBL(g_ahp) DBL(dt) DBL(j_ext)
#undef INT
#undef DBL
  if (!strcmp(key, "rows")) { n->rows = (int32_t)atol(v); return 0; }
  if (!strcmp(key, "cols")) { n->cols = (int32_t)atol(v); return 0; }
  if (!strcmp(key, "seed")) { n->seed = (uint64_t)strtoull(v, NULL, 10); return 0; }
  if (!strcmp(key, "ext_rate_hz")) { n->ext_rate_hz = atof(v); return 0; }
  return -1;
}

static int errors(void) {
  sim_config_t c;
  sim_net_t net;
  sim_t* sim = (sim_t*)&c;  /* must be overwritten with NULL */
  recipe(&c, &net);
  c.npc = 0;
  if (sim_create(&c, NULL, NULL, &sim) != DPSNN_EINVAL || sim != NULL) return fail("npc 0", -99, NULL);
  if (!sim_last_error(NULL)[0]) return fail("empty create error", -99, NULL);
  recipe(&c, &net);
  c.d_max = 40;
  sim_sizes_t sz;
  if (sim_query_sizes(&c, &sz) != DPSNN_EINVAL) return fail("query d_max 40", -99, NULL);
  if (sim_query_sizes(&c, NULL) != DPSNN_EINVAL) return fail("query NULL sizes", -99, NULL);
  if (sim_create(NULL, NULL, NULL, &sim) != DPSNN_EINVAL) return fail("NULL config", -99, NULL);
  if (sim_step(NULL, 1) != DPSNN_EINVAL || sim_sync(NULL) != DPSNN_EINVAL || sim_now(NULL) != -1)
    return fail("NULL handle", -99, NULL);
  sim_destroy(NULL);
  printf("errors ok\n");
  return 0;
}

static int run(int64_t steps, int argc, char** argv) {
  sim_config_t c;
  sim_net_t net;
  recipe(&c, &net);
  for (int a = 0; a < argc; ++a)
    if (set_field(&c, &net, argv[a])) { fprintf(stderr, "bad argument %s\n", argv[a]); return 2; }
  int64_t n = (int64_t)net.rows * net.cols * c.npc;
  c.record_steps = steps;
  c.raster_capacity = steps * n;
  sim_sizes_t sz;
  int rc = sim_query_sizes(&c, &sz);
  if (rc) return fail("sim_query_sizes", rc, NULL);
  if (sz.n_neurons != n || sz.n_records <= 0 || sz.synapse_bytes < 4 * (uint64_t)sz.n_records)
    return fail("sizes", -99, NULL);
  sim_t* sim = NULL;
  rc = sim_create(&c, NULL, NULL, &sim);
  if (rc) return fail("sim_create", rc, NULL);
  rc = sim_step(sim, steps);
  if (rc) return fail("sim_step", rc, sim);
  rc = sim_sync(sim);
  if (rc) return fail("sim_sync", rc, sim);
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(steps + 1));
  int64_t total = 0;
  rc = sim_read_spikes(sim, 0, 0, steps, off, NULL, 0, &total);
  if (rc != DPSNN_OK && rc != DPSNN_ETRUNC) return fail("sim_read_spikes size", rc, sim);
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  rc = sim_read_spikes(sim, 0, 0, steps, off, ids, total, &total);
  if (rc) return fail("sim_read_spikes", rc, sim);
  for (int64_t u = 0; u < steps; ++u) {
    printf("step %lld %lld", (long long)u, (long long)(off[u + 1] - off[u]));
    for (int64_t q = off[u]; q < off[u + 1]; ++q) printf(" %d", ids[q]);
    printf("\n");
  }
  sim_stats_t st;
  rc = sim_get_stats(sim, 0, &st);
  if (rc) return fail("sim_get_stats", rc, sim);
  printf("counts %lld %lld %lld\n", (long long)st.spikes, (long long)st.events_recurrent,
         (long long)st.events_external);
  free(ids);
  free(off);
  sim_destroy(sim);
  return 0;
}

int main(int argc, char** argv) {
  if (argc >= 2 && !strcmp(argv[1], "errors")) return errors();
  if (argc >= 3 && !strcmp(argv[1], "run")) return run(atoll(argv[2]), argc - 3, argv + 3);
  fprintf(stderr, "usage: abi_client errors | run STEPS key=value ...\n");
  return 2;
}
