// autotune.hip -- choose the launch configuration of the step by measurement.
//
// Every candidate (delivery form, workgroup size, tile shape, graph chunk) computes the
// same bits: the input is an integer sum and the float32 update is fixed.  The tuner runs
// each candidate from one saved state for a fixed window, timed with HIP events on the
// simulation's stream, checks that all candidates reach the same state digest, and keeps
// the fastest.  Results may be cached in a JSON-lines file keyed by the device and the
// simulation's shape.
#include <stdio.h>
#include <string.h>

#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "dpsnn_internal.h"

namespace {

constexpr int32_t kTuneSlot = 63;

std::string shape_key(const sim& s) {
  hipDeviceProp_t prop;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch << "|npc" << s.npc << "|nd" << s.nd << "|nets";
  for (const sim_net_t& n : s.nets) k << ":" << n.rows << "x" << n.cols << "@" << n.ext_rate_hz;
  k << "|train" << (s.wfx ? 1 : 0) << "|model" << s.model << "|conn" << s.cfg.conn_kernel
    << "|stdp" << s.cfg.stdp;
  return k.str();
}

bool cache_lookup(const char* path, const std::string& key, sim_launch_t* out, double* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const std::string tag = "\"key\": \"" + key + "\"";
    if (line.find(tag) == std::string::npos) continue;
    sim_launch_t l{};
    double t = 0;
    const char* p = strstr(line.c_str(), "\"delivery\":");
    if (!p || sscanf(p, "\"delivery\": %d, \"block\": %d, \"tile_x\": %d, \"tile_y\": %d, "
                        "\"graph_steps\": %d, \"gather_steps\": %d, \"ms_per_step\": %lf",
                     &l.delivery, &l.block, &l.tile_x, &l.tile_y, &l.graph_steps,
                     &l.gather_steps, &t) != 7)
      continue;
    *out = l;
    *ms = t;
    found = true;  // the last matching line wins
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const sim_launch_t& l, double ms) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{\"key\": \"%s\", \"delivery\": %d, \"block\": %d, \"tile_x\": %d, \"tile_y\": %d, "
          "\"graph_steps\": %d, \"gather_steps\": %d, \"ms_per_step\": %.6f}\n",
          key.c_str(), l.delivery, l.block, l.tile_x, l.tile_y, l.graph_steps, l.gather_steps, ms);
  fclose(f);
}

}  // namespace

extern "C" int sim_autotune(sim_t* s, int32_t window, const char* cache_path, sim_launch_t* best,
                            double* best_ms_per_step) {
  if (!s) return DPSNN_EINVAL;
  if (window < 1) {
    s->err = "window must be >= 1";
    return DPSNN_EINVAL;
  }
  int rc = sim_sync(s);
  if (rc != DPSNN_OK) return rc;
  const std::string key = shape_key(*s);
  sim_launch_t chosen{};
  double chosen_ms = 0;
  if (cache_lookup(cache_path, key, &chosen, &chosen_ms)) {
    rc = sim_set_launch(s, &chosen);
    if (rc == DPSNN_OK) {
      if (best) *best = chosen;
      if (best_ms_per_step) *best_ms_per_step = chosen_ms;
      return DPSNN_OK;
    }
  }
  sim_launch_t original{};
  sim_get_launch(s, &original);
  if ((rc = sim_save(s, kTuneSlot)) != DPSNN_OK) return rc;

  std::vector<sim_launch_t> cands;
  // the arrival form keeps the tiling its synapse store was split for; other tilings read
  // more synapses than they keep, so only the workgroup size, the gather window and graph
  // chunks are searched
  const int blocks[] = {256, 512, 1024};
  for (int b : blocks)
    for (int gw : {1, 2, 4})
      for (int gs : {0, window})
        cands.push_back(sim_launch_t{DPSNN_DELIVERY_ARRIVAL, b, s->native_tx, s->native_ty, gs, gw});
  // the push form scatters with device-scope atomics; only worth trying on small networks
  if (s->n_neurons <= 200000)
    for (int b : {256, 1024})
      for (int gs : {0, window})
        cands.push_back(sim_launch_t{DPSNN_DELIVERY_PUSH, b, original.tile_x, original.tile_y, gs, 1});

  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    s->err = "hipEventCreate failed";
    return DPSNN_EHIP;
  }
  const bool timing = s->timing;
  s->timing = false;
  bool have_ref = false, have_best = false;
  uint64_t ref_digest = 0;
  double best_t = 0;
  sim_launch_t best_l = original;
  std::string mismatch;
  for (const sim_launch_t& c : cands) {
    if (sim_restore(s, kTuneSlot) != DPSNN_OK) break;
    if (sim_set_launch(s, &c) != DPSNN_OK) continue;  // e.g. a tile that does not fit the LDS
    // untimed pass (code loading, graph capture), then the timed pass from the same state
    if (sim_step(s, window) != DPSNN_OK || sim_sync(s) != DPSNN_OK) break;
    if (sim_restore(s, kTuneSlot) != DPSNN_OK) break;
    (void)hipEventRecord(e0, s->stream);
    if (sim_step(s, window) != DPSNN_OK) break;
    (void)hipEventRecord(e1, s->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    uint64_t d = 0;
    if (sim_state_digest(s, &d) != DPSNN_OK) break;
    if (!have_ref) {
      ref_digest = d;
      have_ref = true;
    } else if (d != ref_digest) {
      mismatch = "candidate delivery " + std::to_string(c.delivery) + " block " +
                 std::to_string(c.block) + " tile " + std::to_string(c.tile_x) + "x" +
                 std::to_string(c.tile_y) + " gather " + std::to_string(c.gather_steps) +
                 " reached a different state";
      break;
    }
    if (!have_best || ms < best_t) {
      best_t = ms;
      best_l = c;
      have_best = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->timing = timing;
  rc = sim_restore(s, kTuneSlot);
  if (rc != DPSNN_OK) return rc;
  if (!mismatch.empty()) {
    sim_set_launch(s, &original);
    s->err = "autotune: " + mismatch;
    return DPSNN_ESTATE;
  }
  if (!have_best) {
    sim_set_launch(s, &original);
    s->err = "autotune: no candidate ran";
    return DPSNN_ESTATE;
  }
  rc = sim_set_launch(s, &best_l);
  if (rc != DPSNN_OK) return rc;
  const double per_step = best_t / window;
  cache_store(cache_path, key, best_l, per_step);
  if (best) *best = best_l;
  if (best_ms_per_step) *best_ms_per_step = per_step;
  return DPSNN_OK;
}

// Creation-time choice of the native tiling: each admissible shape is built, settled, timed
// and destroyed in turn (one simulation's device memory at a time); all must agree bit for
// bit (state digest).
extern "C" int sim_tune_tiling(const sim_config_t* cfg, int32_t settle, int32_t window,
                               int32_t* tile_x, int32_t* tile_y, double* ms_per_step) {
  if (!cfg || !tile_x || !tile_y) {
    dpsnn::set_create_error("cfg, tile_x and tile_y are required");
    return DPSNN_EINVAL;
  }
  if (settle < 0 || window < 1) {
    dpsnn::set_create_error("settle must be >= 0 and window >= 1");
    return DPSNN_EINVAL;
  }
  static const int shapes[][2] = {{3, 3}, {3, 2}, {2, 3}, {2, 2}, {2, 1}, {1, 2}, {1, 1}};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    dpsnn::set_create_error("hipEventCreate failed");
    return DPSNN_EHIP;
  }
  bool have = false;
  uint64_t ref = 0;
  double best_ms = 0;
  int bx = 0, by = 0, rc = DPSNN_OK;
  std::string last_refusal = "no tile shape is admissible for this configuration";
  for (const auto& sh : shapes) {
    sim_config_t c = *cfg;
    c.tile_x = sh[0];
    c.tile_y = sh[1];
    c.record_steps = 0;
    c.raster_capacity = 0;
    sim_t* s = nullptr;
    const int crc = sim_create(&c, nullptr, nullptr, &s);
    if (crc == DPSNN_EINVAL || crc == DPSNN_ENOMEM) {
      // the shape does not fit the LDS or the stencil, or its store does not fit the device
      last_refusal = sim_last_error(nullptr);
      (void)hipGetLastError();
      continue;
    }
    if (crc != DPSNN_OK) {
      rc = crc;
      break;
    }
    float ms = 0;
    uint64_t d = 0;
    int src = sim_step(s, settle);
    if (src == DPSNN_OK) src = sim_sync(s);
    if (src == DPSNN_OK) {
      (void)hipEventRecord(e0, s->stream);
      src = sim_step(s, window);
      (void)hipEventRecord(e1, s->stream);
    }
    if (src == DPSNN_OK) src = sim_sync(s);
    if (src == DPSNN_OK) {
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(&ms, e0, e1);
      src = sim_state_digest(s, &d);
    }
    if (src != DPSNN_OK) dpsnn::set_create_error(std::string("tiling ") + std::to_string(sh[0]) +
                                                 "x" + std::to_string(sh[1]) + ": " +
                                                 sim_last_error(s));
    sim_destroy(s);
    if (src != DPSNN_OK) {
      rc = src;
      break;
    }
    if (have && d != ref) {
      dpsnn::set_create_error(std::string("tiling ") + std::to_string(sh[0]) + "x" +
                              std::to_string(sh[1]) + " reached a different state");
      rc = DPSNN_ESTATE;
      break;
    }
    ref = d;
    const double per = (double)ms / window;
    if (!have || per < best_ms) {
      best_ms = per;
      bx = sh[0];
      by = sh[1];
    }
    have = true;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DPSNN_OK) return rc;
  if (!have) {
    dpsnn::set_create_error(last_refusal);
    return DPSNN_EINVAL;
  }
  *tile_x = bx;
  *tile_y = by;
  if (ms_per_step) *ms_per_step = best_ms;
  return DPSNN_OK;
}
