// capi.hip -- host side of libdpsnn: the C ABI declared in include/dpsnn.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "dpsnn_internal.h"

using namespace dpsnn;

namespace {

thread_local std::string g_create_error;

struct Fail {
  int code;
  std::string msg;
};

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw Fail{DPSNN_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};          \
  } while (0)

void* dalloc(sim& s, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Fail{DPSNN_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  s.bufs.push_back(DevBuf{p, bytes});
  s.device_bytes += bytes;
  return p;
}

void dfree(sim& s, void* p) {
  if (!p) return;
  for (size_t q = 0; q < s.bufs.size(); ++q) {
    if (s.bufs[q].p == p) {
      s.device_bytes -= s.bufs[q].bytes;
      (void)hipFree(p);
      s.bufs.erase(s.bufs.begin() + (long)q);
      return;
    }
  }
}

// Caller-owned regions of device memory (sim_buffers_t).  Arrays of a region are carved in
// a fixed order at 256-byte aligned offsets; region_sizes() gives the same layout's sizes.
enum { kRegSyn = 0, kRegIndex = 1, kRegState = 2, kRegHist = 3 };
const char* const kRegionName[4] = {"synapses", "index", "state", "history"};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void* carve(sim& s, int r, size_t bytes) {
  if (!s.region_base[r]) return dalloc(s, bytes);
  const size_t b = align256(bytes ? bytes : 1);
  if (s.region_used[r] + b > s.region_cap[r])
    throw Fail{DPSNN_EINVAL, std::string("the caller's ") + kRegionName[r] +
                                 " buffer is smaller than sim_query_sizes reports"};
  void* p = s.region_base[r] + s.region_used[r];
  s.region_used[r] += b;
  return p;
}

// Sizes of the four regions for a store of `records` synapse records (padding included).
void region_sizes(const sim& s, int64_t records, size_t out[4]) {
  const size_t N = (size_t)s.n_neurons, C = (size_t)s.n_cols, dh = (size_t)s.dh,
               npc = (size_t)s.npc, P = (size_t)s.n_parts, nd = (size_t)s.nd;
  out[kRegSyn] = align256(sizeof(uint32_t) * (size_t)(records + 4));
  out[kRegIndex] = align256(sizeof(int64_t) * (N + 1)) + align256(sizeof(int32_t) * N) +
                   align256((size_t)s.idxw * (size_t)s.n_idx);
  out[kRegState] = 2 * align256(sizeof(float) * N) + align256(N);
  out[kRegHist] = align256(sizeof(int32_t) * dh * C) + align256(sizeof(uint16_t) * dh * C * npc) +
                  align256(sizeof(uint64_t) * dh * P * npc) +
                  align256(sizeof(uint16_t) * dh * P * (nd + 1) * npc);
}

template <typename T>
T* upload(sim& s, const std::vector<T>& h) {
  T* d = (T*)dalloc(s, sizeof(T) * std::max<size_t>(h.size(), 1));
  if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s.stream));
  return d;
}

// Gaussian factor exp(-r^2 / 2 sigma^2) of a stencil offset, r the distance of column centres.
double gauss_factor(const sim_config_t& c, int dy, int dx) {
  const double r2 = (double)(dy * dy + dx * dx) * c.spacing_um * c.spacing_um;
  return exp(-r2 / (2.0 * c.lateral_sigma_um * c.lateral_sigma_um));
}

// Half-width of the stencil: 1 for the 3x3 kernel; for the Gaussian kernel the largest
// axis offset (at most 3) whose factor reaches the cut-off.
int stencil_radius(const sim_config_t& c) {
  if (c.conn_kernel != DPSNN_CONN_GAUSS) return 1;
  int r = 0;
  while (r < 3 && gauss_factor(c, 0, r + 1) >= c.lateral_cutoff) ++r;
  return r;
}

// Probability of one stencil offset (section 2, Methods: connectivity decreasing with the
// distance between columns): the own column; for the 3x3 kernel a neighbour weighted by
// exp(-distance / decay) with the remote share spread over the 8 neighbours; for the
// Gaussian kernel A exp(-r^2 / 2 sigma^2) where that factor reaches the cut-off, else 0.
double offset_prob(const sim_config_t& c, int dy, int dx) {
  if (dy == 0 && dx == 0) return c.p_own;
  if (c.conn_kernel == DPSNN_CONN_GAUSS) {
    const double g = gauss_factor(c, dy, dx);
    return g >= c.lateral_cutoff ? c.lateral_amp * g : 0.0;
  }
  const double edge = exp(-(c.spacing_um / c.decay_um));
  const double diag = exp(-(sqrt(2.0) * c.spacing_um / c.decay_um));
  const double norm = 4.0 * edge + 4.0 * diag;
  const double one = (dy == 0 || dx == 0) ? edge : diag;
  return c.p_remote * one / norm;
}

uint64_t threshold_of(double p) {
  const double t = floor(p * 4294967296.0);
  if (t <= 0.0) return 0;
  if (t >= 4294967296.0) return (uint64_t)1 << 32;
  return (uint64_t)t;
}

// Poisson(lam) inverse-CDF thresholds, floor(F(k) 2^32) capped at 2^32.
void poisson_thresholds(double lam, uint64_t* tab) {
  double pk = exp(-lam);
  double cdf = 0.0;
  for (int k = 0; k < kPoissonEntries; ++k) {
    if (k > 0) pk = pk * lam / (double)k;
    cdf = cdf + pk;
    const double t = floor(cdf * 4294967296.0);
    tab[k] = t >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)t;
  }
}

void validate(const sim_config_t* c) {
  auto bad = [](const std::string& m) { throw Fail{DPSNN_EINVAL, m}; };
  if (!c) bad("config is NULL");
  if (c->npc < 1 || c->npc > kMaxNpc) bad("npc must be in [1, 4096]");
  if (c->n_exc < 0 || c->n_exc > c->npc) bad("n_exc must be in [0, npc]");
  if (c->d_min < 1 || c->d_max < c->d_min || c->d_max > kMaxDelay)
    bad("delays must satisfy 1 <= d_min <= d_max <= 32");
  if (!(c->p_own >= 0 && c->p_own <= 1 && c->p_remote >= 0 && c->p_own + c->p_remote <= 1.0 + 1e-12))
    bad("p_own, p_remote must be probabilities with p_own + p_remote <= 1");
  if (!(c->decay_um > 0 && c->spacing_um > 0)) bad("decay_um and spacing_um must be positive");
  const double lim = 32767.0 / 16384.0;
  if (!(fabs(c->we_mu) + 6 * c->we_sigma < lim && fabs(c->wi_mu) + 6 * c->wi_sigma < lim) ||
      c->we_sigma < 0 || c->wi_sigma < 0)
    bad("weights must satisfy |mu| + 6 sigma < 2 mV (int16 at 2^-14 mV)");
  if (!(c->tau_m > 0 && c->tau_ca > 0 && c->dt > 0)) bad("time constants and dt must be positive");
  if (c->t_ref < 0 || c->t_ref > 255) bad("t_ref must be in [0, 255]");
  if (c->ext_syn < 0) bad("ext_syn must be >= 0");
  if (c->n_nets < 1 || !c->nets) bad("need at least one network");
  if (c->delivery < 0 || c->delivery > 2) bad("unknown delivery strategy");
  if (!(c->block == 0 || c->block == 64 || c->block == 128 || c->block == 256 ||
        c->block == 512 || c->block == 1024))
    bad("block must be 0, 64, 128, 256, 512 or 1024");
  if (c->tile_x < 0 || c->tile_y < 0 || c->tile_x > kMaxTileSide || c->tile_y > kMaxTileSide ||
      ((c->tile_x == 0) != (c->tile_y == 0)))
    bad("tile sides must both be 0 (auto) or both in [1, 4]");
  if (c->record_steps < 0 || c->raster_capacity < 0) bad("raster sizes must be >= 0");
  if (c->train_mode && c->ckpt_every < 1) bad("ckpt_every must be >= 1 in train mode");
  if (c->train_mode && !(c->surrogate_beta > 0)) bad("surrogate_beta must be > 0 in train mode");
  if (c->neuron_model != DPSNN_NEURON_LIF && c->neuron_model != DPSNN_NEURON_IZHIKEVICH)
    bad("unknown neuron_model");
  if (c->neuron_model == DPSNN_NEURON_LIF && c->g_na != 0.0 && !(c->tau_na > 0))
    bad("tau_na must be positive when g_na != 0");
  if (c->neuron_model == DPSNN_NEURON_IZHIKEVICH &&
      !(std::isfinite(c->izh_vpeak) && std::isfinite(c->izh_a_e) && std::isfinite(c->izh_b_e) &&
        std::isfinite(c->izh_c_e) && std::isfinite(c->izh_d_e) && std::isfinite(c->izh_a_i) &&
        std::isfinite(c->izh_b_i) && std::isfinite(c->izh_c_i) && std::isfinite(c->izh_d_i)))
    bad("Izhikevich parameters must be finite");
  if (c->conn_kernel != DPSNN_CONN_EXP3X3 && c->conn_kernel != DPSNN_CONN_GAUSS)
    bad("unknown conn_kernel");
  if (c->conn_kernel == DPSNN_CONN_GAUSS &&
      !(c->lateral_sigma_um > 0 && c->lateral_cutoff > 0 && c->lateral_cutoff <= 1 &&
        c->lateral_amp >= 0 && c->lateral_amp <= 1))
    bad("Gaussian kernel needs lateral_sigma_um > 0, 0 < lateral_cutoff <= 1 and "
        "0 <= lateral_amp <= 1");
  if (c->train_mode && (c->neuron_model != DPSNN_NEURON_LIF || c->g_na != 0.0))
    bad("train mode needs the LIF neuron with g_na = 0 (the adjoint of the other models is not "
        "defined)");
  if (c->stdp) {
    if (!(c->stdp_tau_plus > 0 && c->stdp_tau_minus > 0 && std::isfinite(c->stdp_tau_plus) &&
          std::isfinite(c->stdp_tau_minus)))
      bad("stdp_tau_plus and stdp_tau_minus must be positive");
    if (!(c->stdp_w_max > 0 && c->stdp_w_max < 2.0)) bad("stdp_w_max must be in (0, 2) mV");
    // a trace never exceeds 1 / (1 - exp(-dt / tau)): the largest change must fit an int32
    const double xp = 1.0 / (1.0 - exp(-c->dt / c->stdp_tau_plus));
    const double xm = 1.0 / (1.0 - exp(-c->dt / c->stdp_tau_minus));
    if (!(c->stdp_a_plus >= 0 && c->stdp_a_minus >= 0 &&
          c->stdp_a_plus * 16384.0 * xp < 1073741824.0 &&
          c->stdp_a_minus * 16384.0 * xm < 1073741824.0))
      bad("stdp_a_plus and stdp_a_minus must be >= 0 with a * 2^14 / (1 - exp(-dt / tau)) "
          "< 2^30");
    if (c->train_mode) bad("STDP and train mode exclude each other");
    if (c->delivery == DPSNN_DELIVERY_PUSH) bad("STDP needs the arrival form");
  }
  int64_t cols = 0;
  for (int n = 0; n < c->n_nets; ++n) {
    const sim_net_t& t = c->nets[n];
    if (t.rows < 1 || t.cols < 1) bad("grid sides must be >= 1");
    if (!(t.ext_rate_hz >= 0)) bad("ext_rate_hz must be >= 0");
    const double lam = (double)c->ext_syn * t.ext_rate_hz * c->dt * 1e-3;
    if (lam > 20.0) bad("external mean count per step must be <= 20 (Poisson table cap 63)");
    cols += (int64_t)t.rows * t.cols;
  }
  if (cols * c->npc >= ((int64_t)1 << 31)) bad("total neurons must be < 2^31");
  if (c->stdp && (cols * c->npc >= ((int64_t)1 << 24) || cols > 16000))
    bad("STDP needs fewer than 2^24 neurons and at most 16000 columns");
  if (cols * (c->d_max + 1) * c->npc >= ((int64_t)1 << 31)) bad("spike history exceeds 2^31 entries");
}

// Default workgroup size: the tile kernel uses 1024 threads (one workgroup per CU holds a
// 4x4 tile's accumulators), the per-column push kernels 256.
int32_t default_block(int32_t delivery) { return delivery == DPSNN_DELIVERY_PUSH ? 256 : 1024; }

void set_constants(sim& s) {
  const sim_config_t& c = s.cfg;
  s.nk.pm = (float)exp(-c.dt / c.tau_m);
  s.nk.pc = (float)exp(-c.dt / c.tau_ca);
  s.nk.gam = (float)(c.g_ahp * c.dt);
  s.nk.alpha = (float)c.ca_inc;
  s.nk.theta = (float)c.theta;
  s.nk.vreset = (float)c.v_reset;
  s.nk.jfx = (int32_t)rint(c.j_ext * 65536.0);
  s.nk.tref = c.t_ref;
  s.nk.pna = c.tau_na > 0 ? (float)exp(-c.dt / c.tau_na) : 0.0f;
  s.nk.gna = (float)(c.g_na * c.dt);
  s.nk.alpha_na = (float)c.na_inc;
  s.nk.vpeak = (float)c.izh_vpeak;
  const double ia[2] = {c.izh_a_e, c.izh_a_i}, ib[2] = {c.izh_b_e, c.izh_b_i},
               ic[2] = {c.izh_c_e, c.izh_c_i}, id[2] = {c.izh_d_e, c.izh_d_i};
  for (int t = 0; t < 2; ++t) {
    s.nk.ia[t] = (float)ia[t];
    s.nk.ib[t] = (float)ib[t];
    s.nk.ic[t] = (float)ic[t];
    s.nk.id[t] = (float)id[t];
  }
  s.model = c.neuron_model == DPSNN_NEURON_IZHIKEVICH ? kModelIzh
            : c.g_na != 0.0                           ? kModelLifNa
                                                      : kModelLif;
  if (s.model == kModelIzh) s.nk.tref = 0;  // no refractory period
}

// Compute units of the current device (256 on an MI355X when the query fails).
static int device_cu_count() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
      prop.multiProcessorCount > 0)
    return prop.multiProcessorCount;
  return 256;
}

// Round-robin merge of per-XCD work lists (-1 where a list ran out).
std::vector<int32_t> interleave(const std::vector<std::vector<int32_t>>& lanes) {
  size_t longest = 0;
  for (const auto& L : lanes) longest = std::max(longest, L.size());
  std::vector<int32_t> order;
  for (size_t q = 0; q < longest; ++q)
    for (size_t x = 0; x < lanes.size(); ++x) order.push_back(q < lanes[x].size() ? lanes[x][q] : -1);
  return order;
}

void release(sim& s, void* p) {
  if (!p) return;
  for (size_t q = 0; q < s.bufs.size(); ++q) {
    if (s.bufs[q].p == p) {
      s.device_bytes -= s.bufs[q].bytes;
      (void)hipFree(p);
      s.bufs.erase(s.bufs.begin() + (long)q);
      return;
    }
  }
}

// Native tile (x, y index) of a column of network n under a tx x ty tiling (clamped to the
// network's grid; edge tiles are smaller).
static void tile_of(const sim& s, int n, int tx, int ty, int cl, int* txi, int* tyi) {
  const int rows = s.nets[n].rows, cols = s.nets[n].cols;
  const int ttx = std::min(tx, cols), tty = std::min(ty, rows);
  (void)rows;
  *txi = (cl % cols) / ttx;
  *tyi = (cl / cols) / tty;
}

bool compute_parts(const sim& s, int tx, int ty, std::vector<int32_t>& part,
                   std::vector<int32_t>& np, std::vector<int32_t>& prank);

// Can a tx x ty tiling be the native one: parts within their limits for this stencil?
bool parts_fit(const sim& s, int tx, int ty) {
  std::vector<int32_t> part, np, prank;
  return compute_parts(s, tx, ty, part, np, prank);
}

// Does a tx x ty tiling fit the LDS of the tile kernel?
bool tile_fits(sim& s, int tx, int ty) {
  if (tx < 1 || ty < 1 || tx > kMaxTileSide || ty > kMaxTileSide) return false;
  int maxc = 0;
  for (int n = 0; n < s.n_nets; ++n)
    maxc = std::max(maxc, std::min(tx, s.nets[n].cols) * std::min(ty, s.nets[n].rows));
  const int32_t old = s.tile_max_cols;
  s.tile_max_cols = maxc;
  const bool ok = tile_lds_ok(s);
  s.tile_max_cols = old;
  return ok;
}

// Parts of every source column under a tx x ty tiling: the stencil ranks whose target
// columns lie in one tile form one part, parts numbered by first appearance in rank order;
// prank is the rank of each column inside its part.  Returns false when a part would hold
// more than kMaxPartCols columns or a column more than kMaxParts parts.
bool compute_parts(const sim& s, int tx, int ty, std::vector<int32_t>& part,
                   std::vector<int32_t>& np, std::vector<int32_t>& prank) {
  part.assign((size_t)s.n_cols * kMaxNbr, -1);
  prank.assign((size_t)s.n_cols * kMaxNbr, -1);
  np.assign((size_t)s.n_cols, 0);
  for (int n = 0; n < s.n_nets; ++n) {
    for (int cl = 0; cl < s.nets[n].rows * s.nets[n].cols; ++cl) {
      const int32_t g = s.net_col0[n] + cl;
      std::vector<int> seen, size;
      for (int r = 0; r < s.h_nn[g]; ++r) {
        const int32_t t = s.h_nbr[(size_t)g * kMaxNbr + r] - s.net_col0[n];
        int xi, yi;
        tile_of(s, n, tx, ty, t, &xi, &yi);
        const int key = yi * 65536 + xi;
        int p = -1;
        for (size_t q = 0; q < seen.size(); ++q)
          if (seen[q] == key) p = (int)q;
        if (p < 0) {
          p = (int)seen.size();
          seen.push_back(key);
          size.push_back(0);
        }
        part[(size_t)g * kMaxNbr + r] = p;
        prank[(size_t)g * kMaxNbr + r] = size[p]++;
        if (size[p] > kMaxPartCols) return false;
      }
      if ((int)seen.size() > kMaxParts) return false;
      np[g] = (int32_t)seen.size();
    }
  }
  return true;
}

void build_parts(sim& s, int tx, int ty) {
  std::vector<int32_t> part, np, prank;
  if (!compute_parts(s, tx, ty, part, np, prank))
    throw Fail{DPSNN_EINVAL, "the tiling gives a part of more than 9 columns or a column of "
                             "more than 16 parts for this stencil"};
  std::vector<int64_t> pbase((size_t)s.n_cols + 1, 0);
  std::vector<int32_t> pfirst((size_t)s.n_cols + 1, 0);
  for (int32_t g = 0; g < s.n_cols; ++g) {
    pbase[g + 1] = pbase[g] + (int64_t)s.npc * np[g];
    pfirst[g + 1] = pfirst[g] + np[g];
  }
  s.n_parts = pfirst[s.n_cols];
  // the columns of every part by rank, and their stencil ranks
  std::vector<int32_t> pcol((size_t)std::max(s.n_parts, 1) * kMaxPartCols, -1),
      psrank((size_t)std::max(s.n_parts, 1) * kMaxPartCols, -1);
  for (int32_t g = 0; g < s.n_cols; ++g)
    for (int r = 0; r < s.h_nn[g]; ++r) {
      const size_t e = (size_t)(pfirst[g] + part[(size_t)g * kMaxNbr + r]) * kMaxPartCols +
                       prank[(size_t)g * kMaxNbr + r];
      pcol[e] = s.h_nbr[(size_t)g * kMaxNbr + r];
      psrank[e] = r;
    }
  s.col_pfirst = upload(s, pfirst);
  s.h_part = part;
  s.h_np = np;
  s.h_prank = prank;
  s.n_idx = pbase[s.n_cols];
  s.native_tx = tx;
  s.native_ty = ty;
  s.col_part = upload(s, part);
  s.col_prank = upload(s, prank);
  s.col_np = upload(s, np);
  s.col_pbase = upload(s, pbase);
  s.part_col = upload(s, pcol);
  s.part_srank = upload(s, psrank);
}

// Tiles of tx x ty target columns (clamped to each network's grid; edge tiles are smaller).
// For each tile: its columns, every (source column, part) with synapses into it, and per
// pair the tile slot of each rank of the part.  Tiles are ordered like the columns: strips
// of each network per XCD.
void set_tile_bases(sim& s);

void build_tiles(sim& s, int tx, int ty) {
  if (tx < 1 || ty < 1 || tx > kMaxTileSide || ty > kMaxTileSide)
    throw Fail{DPSNN_EINVAL, "tile sides must be in [1, 4]"};
  std::vector<int32_t> cinfo, tncols, pinfo, tnet, npairs;
  std::vector<int32_t> pfirst((size_t)s.n_cols + 1, 0);
  for (int32_t g = 0; g < s.n_cols; ++g) pfirst[g + 1] = pfirst[g] + s.h_np[g];
  std::vector<uint64_t> tslots;
  std::vector<int32_t> tsrc, tsrc_off(1, 0);
  std::vector<std::vector<int32_t>> lanes(8);
  int rot = 0, maxc = 0;
  for (int n = 0; n < s.n_nets; ++n) {
    const int rows = s.nets[n].rows, cols = s.nets[n].cols;
    const int ttx = std::min(tx, cols), tty = std::min(ty, rows);
    const int ntx = (cols + ttx - 1) / ttx, nty = (rows + tty - 1) / tty;
    const int nstrip = std::min(8, ntx);
    for (int st = 0; st < nstrip; ++st) {
      const int a0 = st * ntx / nstrip, a1 = (st + 1) * ntx / nstrip;
      for (int yi = 0; yi < nty; ++yi) {
        for (int xi = a0; xi < a1; ++xi) {
          std::vector<int32_t> tc;
          for (int y = yi * tty; y < std::min(rows, (yi + 1) * tty); ++y)
            for (int x = xi * ttx; x < std::min(cols, (xi + 1) * ttx); ++x)
              tc.push_back(s.net_col0[n] + y * cols + x);
          std::vector<int32_t> src;
          for (int32_t g : tc)
            for (int r = 0; r < s.h_nn[g]; ++r) src.push_back(s.h_nbr[(size_t)g * kMaxNbr + r]);
          std::sort(src.begin(), src.end());
          src.erase(std::unique(src.begin(), src.end()), src.end());
          tsrc.insert(tsrc.end(), src.begin(), src.end());
          tsrc_off.push_back((int32_t)tsrc.size());
          // the source columns of the tile are the columns whose neighbourhood meets it
          // (the stencil is symmetric); each contributes the parts that reach the tile
          std::vector<std::pair<int32_t, int32_t>> pairs;
          std::vector<uint64_t> packs;
          for (int32_t sc : src) {
            for (int p = 0; p < s.h_np[sc]; ++p) {
              // 5-bit field q: the tile slot of the part's column of rank q; every field
              // starts at 31 ("not in the tile"), ranks >= 9 (dummies) keep it
              uint64_t packed = ~(uint64_t)0;
              bool any = false;
              for (int r = 0; r < s.h_nn[sc]; ++r) {
                if (s.h_part[(size_t)sc * kMaxNbr + r] != p) continue;
                const int32_t t = s.h_nbr[(size_t)sc * kMaxNbr + r];
                const int q = s.h_prank[(size_t)sc * kMaxNbr + r];
                for (size_t z = 0; z < tc.size(); ++z)
                  if (tc[z] == t) {
                    packed &= ~((uint64_t)31 << (5 * q));
                    packed |= (uint64_t)z << (5 * q);
                    any = true;
                  }
              }
              if (any) {
                pairs.push_back({sc, p});
                packs.push_back(packed);
              }
            }
          }
          if ((int)tc.size() > kMaxTileCols || (int)pairs.size() > kMaxTilePairs)
            throw Fail{DPSNN_EINVAL, "tile too large"};
          const int32_t id = (int32_t)tncols.size();
          maxc = std::max(maxc, (int)tc.size());
          tncols.push_back((int32_t)tc.size());
          npairs.push_back((int32_t)pairs.size());
          tnet.push_back(n);
          for (int q = 0; q < kMaxTileCols; ++q) {
            const bool in = q < (int)tc.size();
            cinfo.push_back(in ? tc[q] : -1);
            cinfo.push_back(in ? tc[q] - s.net_col0[n] : 0);
            cinfo.push_back(in ? s.h_np[tc[q]] : 0);
            cinfo.push_back(in ? pfirst[tc[q]] : 0);
          }
          for (int q = 0; q < kMaxTilePairs; ++q) {
            const bool in = q < (int)pairs.size();
            pinfo.push_back(in ? pairs[q].first : -1);
            pinfo.push_back(in ? pfirst[pairs[q].first] + pairs[q].second : 0);
            tslots.push_back(in ? packs[q] : ~(uint64_t)0);
          }
          lanes[(st + rot) % 8].push_back(id);
        }
      }
    }
    rot = (rot + nstrip) % 8;
  }
  const int32_t old_max = s.tile_max_cols, old_gk = s.gk;
  s.tile_max_cols = maxc;
  s.gk = 1;  // the fit of one accumulator; the gather window is chosen afterwards
  const bool fits = tile_lds_ok(s);
  s.gk = old_gk;
  if (!fits) {
    s.tile_max_cols = old_max;
    throw Fail{DPSNN_EINVAL, "tile accumulators exceed the 160 KB LDS of a workgroup"};
  }
  release(s, s.tile_order);
  release(s, s.tile_cinfo);
  release(s, s.tile_ncols);
  release(s, s.tile_pinfo);
  release(s, s.tile_net);
  release(s, s.tile_npairs);
  release(s, s.tile_slots);
  release(s, s.tile_work);
  release(s, s.tile_base);
  s.tile_base = nullptr;
  const std::vector<int32_t> order = interleave(lanes);
  s.tile_x = tx;
  s.tile_y = ty;
  s.n_tiles = (int32_t)tncols.size();
  s.grid_tiles = (int32_t)order.size();
  s.tile_order = upload(s, order);
  s.tile_cinfo = upload(s, cinfo);
  s.tile_ncols = upload(s, tncols);
  s.tile_pinfo = upload(s, pinfo);
  s.tile_net = upload(s, tnet);
  s.tile_npairs = upload(s, npairs);
  s.tile_slots = upload(s, tslots);
  s.tile_work = upload(s, std::vector<uint32_t>((size_t)s.n_tiles, 0u));
  s.h_tile_src = tsrc;
  s.h_tile_src_off = tsrc_off;
  // when every tile has its own compute unit the order does not matter
  s.order_by_work = s.n_tiles > device_cu_count();
  if (!s.h_colstart.empty()) set_tile_bases(s);
}

// Per tile, the first 16-byte piece of its source columns' rows; every piece the tile reads
// must lie within 2^32 pieces of it (the folded row order keeps a tile's sources within a
// few grid rows of columns).
void set_tile_bases(sim& s) {
  std::vector<int64_t> base((size_t)s.n_tiles);
  for (int32_t t = 0; t < s.n_tiles; ++t) {
    int64_t lo = INT64_MAX, hi = 0;
    for (int32_t q = s.h_tile_src_off[t]; q < s.h_tile_src_off[t + 1]; ++q) {
      lo = std::min(lo, s.h_colstart[s.h_tile_src[q]]);
      hi = std::max(hi, s.h_colend[s.h_tile_src[q]]);
    }
    if (lo > hi) lo = hi = 0;
    base[t] = lo >> 2;
    if ((hi >> 2) - base[t] >= ((int64_t)1 << 32))
      throw Fail{DPSNN_EINVAL, "the rows of one tile's source columns span more than 2^34 "
                               "records"};
  }
  release(s, s.tile_base);
  s.tile_base = upload(s, base);
}

// After the count pass: move the columns' rows into folded row order (per network, grid rows
// 0, R-1, 1, R-2, ...), so that the rows of stencil neighbours, across the wrap of the torus
// too, lie near each other; record every column's range for the tiles' piece bases.
void fold_rows(sim& s) {
  const int32_t C = s.n_cols;
  std::vector<int64_t> old_start((size_t)C + 1);
  HIPCHK(hipMemcpy2D(old_start.data(), sizeof(int64_t), s.row_base,
                     sizeof(int64_t) * (size_t)s.npc, sizeof(int64_t), (size_t)C + 1,
                     hipMemcpyDeviceToHost));
  std::vector<int64_t> new_start((size_t)C);
  int64_t at = 0;
  for (int n = 0; n < s.n_nets; ++n) {
    const int rows = s.nets[n].rows, cols = s.nets[n].cols;
    for (int pos = 0; pos < rows; ++pos) {
      const int y = (pos & 1) ? rows - 1 - pos / 2 : pos / 2;
      for (int x = 0; x < cols; ++x) {
        const int32_t g = s.net_col0[n] + y * cols + x;
        new_start[g] = at;
        at += old_start[(size_t)g + 1] - old_start[g];
      }
    }
  }
  s.h_colstart = new_start;
  s.h_colend.resize((size_t)C);
  for (int32_t g = 0; g < C; ++g) s.h_colend[g] = new_start[g] + (old_start[(size_t)g + 1] - old_start[g]);
  int64_t* d_old = upload(s, old_start);
  int64_t* d_new = upload(s, new_start);
  HIPCHK(launch_fold_rows(s, d_old, d_new));
  HIPCHK(hipStreamSynchronize(s.stream));
  dfree(s, d_new);
  dfree(s, d_old);
  release(s, s.col_end);
  s.col_end = upload(s, s.h_colend);
}

int64_t tile_count(const sim& s, int tx, int ty) {
  int64_t n = 0;
  for (const sim_net_t& t : s.nets) {
    const int ttx = std::min(tx, t.cols), tty = std::min(ty, t.rows);
    n += (int64_t)((t.cols + ttx - 1) / ttx) * ((t.rows + tty - 1) / tty);
  }
  return n;
}

// Native tiling: the configured one, else the first of the shapes below whose accumulators
// fit the LDS and that gives at least two tiles per compute unit (else the smallest that
// fits: small networks need every workgroup they can get; with one tile per unit the
// uneven tiles leave units idle: 24x24 steps 5 % faster with 1x1 tiles than with 2x1).  3x3
// comes first: with 1240-neuron columns it leaves room for three gather accumulators, and
// 96x96 gives 1024 tiles, four full waves of 256 workgroups.
void choose_native(sim& s, int tx, int ty) {
  if (tx || ty) {
    if (!tile_fits(s, tx, ty)) throw Fail{DPSNN_EINVAL, "tile sides must be in [1, 4] and fit the LDS"};
    if (!parts_fit(s, tx, ty))
      throw Fail{DPSNN_EINVAL, "this tiling gives parts of more than 9 columns or columns of "
                               "more than 16 parts for the stencil"};
    s.native_tx = tx;
    s.native_ty = ty;
    return;
  }
  const int n_cu = device_cu_count();
  static const int shapes[][2] = {{3, 3}, {3, 2}, {2, 2}, {2, 1}, {1, 1}};
  int last = -1;
  for (int q = 0; q < 5; ++q) {
    if (!tile_fits(s, shapes[q][0], shapes[q][1]) || !parts_fit(s, shapes[q][0], shapes[q][1]))
      continue;
    last = q;
    if (tile_count(s, shapes[q][0], shapes[q][1]) >= 2 * (int64_t)n_cu) break;
  }
  if (last < 0) throw Fail{DPSNN_EINVAL, "no tile shape fits the LDS and the stencil"};
  s.native_tx = shapes[last][0];
  s.native_ty = shapes[last][1];
}

// Arrival form: the saved accumulators are derived from the spike history; anything that
// changes the history, the weights or the delivery makes them stale.
void invalidate_gather(sim& s) {
  if (s.d_gath) HIPCHK(hipMemsetAsync(s.d_gath, 0xff, sizeof(int64_t), s.stream));
}

constexpr int kMaxGather = 8;
constexpr int kAutoGather = 4;

// Steps gathered per window: the requested number (0: the largest that fits, at most
// kAutoGather), reduced until the accumulators fit the LDS.
void set_gather(sim& s, int want) {
  if (want < 0 || want > kMaxGather) throw Fail{DPSNN_EINVAL, "gather_steps must be in [0, 8]"};
  if (s.cfg.stdp && want > 1)
    throw Fail{DPSNN_EINVAL, "with STDP every step gathers its own input (gather_steps 0 or 1)"};
  const int old = s.gk;
  int k = want ? want : (s.cfg.stdp ? 1 : kAutoGather);
  for (; k > 1; --k) {
    s.gk = k;
    if (tile_lds_ok(s)) break;
  }
  if (want && k != want) {
    s.gk = old;
    throw Fail{DPSNN_EINVAL, "gather_steps accumulators exceed the LDS"};
  }
  s.gk = k;
  release(s, s.acc_save);
  s.acc_save = nullptr;
  if (k > 1) s.acc_save = (int32_t*)dalloc(s, sizeof(int32_t) * (size_t)k * (size_t)s.n_neurons);
  s.gather_req = want;
  invalidate_gather(s);
}

void build_tables(sim& s) {
  const sim_config_t& c = s.cfg;
  s.net_col0.assign(1, 0);
  for (const sim_net_t& t : s.nets) s.net_col0.push_back(s.net_col0.back() + t.rows * t.cols);
  s.n_cols = s.net_col0.back();
  s.n_neurons = (int64_t)s.n_cols * s.npc;
  std::vector<int32_t> col_net(s.n_cols), col_local(s.n_cols), nn(s.n_cols);
  std::vector<int32_t> nbr((size_t)s.n_cols * kMaxNbr, -1);
  std::vector<uint64_t> thr((size_t)s.n_cols * kMaxNbr, 0);
  for (int n = 0; n < s.n_nets; ++n) {
    const int rows = s.nets[n].rows, cols = s.nets[n].cols;
    for (int cl = 0; cl < rows * cols; ++cl) {
      const int32_t g = s.net_col0[n] + cl;
      col_net[g] = n;
      col_local[g] = cl;
      const int y = cl / cols, x = cl % cols;
      // distinct target columns, probabilities summed in stencil order (dy outer, dx
      // inner); the Gaussian kernel's offsets beyond the cut-off are not in the stencil
      std::vector<std::pair<int, double>> tg;
      const int R = stencil_radius(c);
      for (int dy = -R; dy <= R; ++dy) {
        for (int dx = -R; dx <= R; ++dx) {
          const int ty = ((y + dy) % rows + rows) % rows;
          const int tx = ((x + dx) % cols + cols) % cols;
          const int tcl = ty * cols + tx;
          const double p = offset_prob(c, dy, dx);
          if (c.conn_kernel == DPSNN_CONN_GAUSS && p <= 0.0 && !(dy == 0 && dx == 0)) continue;
          auto it = std::find_if(tg.begin(), tg.end(), [&](const std::pair<int, double>& e) {
            return e.first == tcl;
          });
          if (it == tg.end()) tg.push_back({tcl, 0.0 + p});
          else it->second = it->second + p;
        }
      }
      std::sort(tg.begin(), tg.end());
      nn[g] = (int32_t)tg.size();
      s.max_nn = std::max(s.max_nn, nn[g]);
      for (size_t r = 0; r < tg.size(); ++r) {
        nbr[(size_t)g * kMaxNbr + r] = s.net_col0[n] + tg[r].first;
        thr[(size_t)g * kMaxNbr + r] = threshold_of(tg[r].second);
      }
    }
  }
  // Workgroup order of the per-column kernels.  Workgroups are dealt to the 8 XCDs (each
  // with its own L2) in round-robin order of their index; columns are ordered so that
  // workgroup b lands on XCD b % 8 next to its spatial neighbours (vertical strips of each
  // network, walked row by row).  Slots left over when strips differ in size are -1.
  // A scheduling hint only: any order gives the same results.
  {
    std::vector<std::vector<int32_t>> lanes(8);
    int rot = 0;
    for (int n = 0; n < s.n_nets; ++n) {
      const int rows = s.nets[n].rows, cols = s.nets[n].cols;
      const int nstrip = std::min(8, cols);
      for (int st = 0; st < nstrip; ++st) {
        const int x0 = st * cols / nstrip, x1 = (st + 1) * cols / nstrip;
        std::vector<int32_t>& L = lanes[(st + rot) % 8];
        for (int y = 0; y < rows; ++y)
          for (int x = x0; x < x1; ++x) L.push_back(s.net_col0[n] + y * cols + x);
      }
      rot = (rot + nstrip) % 8;
    }
    std::vector<int32_t> order = interleave(lanes);
    s.grid_cols = (int32_t)order.size();
    s.col_order = upload(s, order);
  }
  s.h_nbr = nbr;
  s.h_nn = nn;
  std::vector<uint32_t> key(2 * (size_t)s.n_nets);
  std::vector<uint64_t> ptab((size_t)s.n_nets * kPoissonEntries);
  for (int n = 0; n < s.n_nets; ++n) {
    key[2 * n] = (uint32_t)(s.nets[n].seed & 0xffffffffu);
    key[2 * n + 1] = (uint32_t)(s.nets[n].seed >> 32);
    const double lam = (double)c.ext_syn * s.nets[n].ext_rate_hz * c.dt * 1e-3;
    poisson_thresholds(lam, &ptab[(size_t)n * kPoissonEntries]);
  }
  s.col_net = upload(s, col_net);
  s.col_local = upload(s, col_local);
  s.col_nn = upload(s, nn);
  s.col_nbr = upload(s, nbr);
  s.col_thr = upload(s, thr);
  s.net_key = upload(s, key);
  s.net_ptab = upload(s, ptab);
}

// Count pass of the generator: records of every row (padding included) and their prefix in
// row_base; returns the store's size in records.
int64_t count_records(sim& s, int64_t** part_out, int64_t* plen_out) {
  const int64_t N = s.n_neurons;
  int32_t* row_len = (int32_t*)dalloc(s, sizeof(int32_t) * (size_t)N);
  s.row_base = (int64_t*)carve(s, kRegIndex, sizeof(int64_t) * (size_t)(N + 1));
  s.deg = (int32_t*)carve(s, kRegIndex, sizeof(int32_t) * (size_t)N);
  const int64_t plen = scan_scratch_len(N);
  int64_t* part = (int64_t*)dalloc(s, sizeof(int64_t) * (size_t)plen);
  HIPCHK(launch_gen_count(s, 0, N, row_len));
  HIPCHK(launch_scan_rows(s, row_len, N, s.row_base, part, plen));
  fold_rows(s);
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, s.row_base + N, sizeof(int64_t), hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  dfree(s, row_len);
  *part_out = part;
  *plen_out = plen;
  return total;
}

void generate(sim& s) {
  const int64_t N = s.n_neurons;
  int64_t* part = nullptr;
  int64_t plen = 0;
  const int64_t total = count_records(s, &part, &plen);
  size_t need[4];
  region_sizes(s, total, need);
  for (int r = 0; r < 4; ++r)
    if (s.region_base[r] && s.region_cap[r] < need[r])
      throw Fail{DPSNN_EINVAL, std::string("the caller's ") + kRegionName[r] + " buffer holds " +
                                   std::to_string(s.region_cap[r]) + " bytes, the simulation needs " +
                                   std::to_string(need[r])};
  // one spare uint4 after the last synapse: the delivery kernels may load whole 16-byte
  // words that straddle the end of a segment
  s.syn = (uint32_t*)carve(s, kRegSyn, sizeof(uint32_t) * (size_t)(total + 4));
  s.idx = (uint8_t*)carve(s, kRegIndex, (size_t)s.idxw * (size_t)s.n_idx);
  HIPCHK(hipMemsetAsync(s.syn + total, 0, 4 * sizeof(uint32_t), s.stream));
  HIPCHK(launch_gen_fill(s, 0, N));
  // the number of synapses (without the padding): scan of the out-degrees
  int64_t* degscan = (int64_t*)dalloc(s, sizeof(int64_t) * (size_t)(N + 1));
  HIPCHK(launch_scan_rows(s, s.deg, N, degscan, part, plen));
  HIPCHK(hipMemcpyAsync(&s.n_syn, degscan + N, sizeof(int64_t), hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  s.n_syn_padded = total;
  s.net_syn0.assign((size_t)s.n_nets + 1, 0);
  for (int n = 0; n <= s.n_nets; ++n) {
    const int64_t i = (int64_t)s.net_col0[n] * s.npc;
    HIPCHK(hipMemcpy(&s.net_syn0[n], degscan + i, sizeof(int64_t), hipMemcpyDeviceToHost));
  }
  if (s.cfg.train_mode) s.canon_start = degscan;  // canonical order of the weights
  else dfree(s, degscan);
  dfree(s, part);
  set_tile_bases(s);
}

void ensure_ring(sim& s) {
  if (s.ring) return;
  const size_t bytes = sizeof(int32_t) * (size_t)s.dh * (size_t)s.n_neurons;
  s.ring = (int32_t*)dalloc(s, bytes);
  HIPCHK(hipMemsetAsync(s.ring, 0, bytes, s.stream));
}

// Materialise the push ring from the spike history (switching from arrival to push).
void ring_from_history(sim& s) {
  ensure_ring(s);
  const size_t nall = (size_t)s.n_neurons;
  for (int n = 0; n < s.n_nets; ++n) {
    // the view is per network: targets relative to the network's first column
    const int32_t g0 = s.net_col0[n], g1 = s.net_col0[n + 1];
    const size_t nn = (size_t)(g1 - g0) * s.npc;
    int32_t* tmp = (int32_t*)dalloc(s, sizeof(int32_t) * (size_t)s.dh * nn);
    HIPCHK(hipMemsetAsync(tmp, 0, sizeof(int32_t) * (size_t)s.dh * nn, s.stream));
    HIPCHK(launch_pend_view(s, tmp, g0, g1));
    for (int q = 0; q < s.dh; ++q) {
      const int64_t slot = (s.now + q) % s.dh;
      HIPCHK(hipMemcpyAsync(s.ring + slot * (int64_t)nall + (int64_t)g0 * s.npc, tmp + q * nn,
                            sizeof(int32_t) * nn, hipMemcpyDeviceToDevice, s.stream));
    }
    HIPCHK(hipStreamSynchronize(s.stream));
    dfree(s, tmp);
  }
}

// The dynamic state saved by a snapshot.  The push ring is not part of it: it is rebuilt
// from the spike history on restore.
constexpr int kSnapParts = 11;

void snapshot_parts(sim& s, size_t* parts, void** ptrs) {
  const size_t N = (size_t)s.n_neurons;
  // plasticity: the weights (the whole store) and the traces
  const bool sp = s.cfg.stdp != 0;
  parts[8] = sp ? sizeof(uint32_t) * (size_t)(s.n_syn_padded + 4) : 0;   ptrs[8] = s.syn;
  parts[9] = sp ? sizeof(float) * N : 0;                              ptrs[9] = s.sp_y;
  parts[10] = sp ? sizeof(float) * (size_t)s.dh * N : 0;              ptrs[10] = s.sp_x;
  parts[7] = s.na ? sizeof(float) * N : 0;                         ptrs[7] = s.na;
  parts[6] = sizeof(unsigned long long) * (size_t)s.n_cols;         ptrs[6] = s.col_spk;
  parts[0] = sizeof(float) * N;                                    ptrs[0] = s.v;
  parts[1] = sizeof(float) * N;                                    ptrs[1] = s.ca;
  parts[2] = N;                                                    ptrs[2] = s.ref;
  parts[3] = sizeof(int32_t) * (size_t)s.dh * s.n_cols;            ptrs[3] = s.hist_cnt;
  parts[4] = sizeof(uint16_t) * (size_t)s.dh * s.n_cols * s.npc;   ptrs[4] = s.hist_ids;
  parts[5] = sizeof(unsigned long long) * kCounters * (size_t)s.n_nets;    ptrs[5] = s.net_cnt;
}

void save_into_ckpt(sim& s, size_t m);

// Plasticity: zero traces and the index of the plastic synapses into each neuron (a count
// per target, its scan, then every record written at its target's next free place).
void setup_stdp(sim& s) {
  const size_t N = (size_t)s.n_neurons;
  if (s.n_syn_padded + 4 > ((int64_t)1 << 35))
    throw Fail{DPSNN_EINVAL, "STDP needs fewer than 2^35 synapse records"};
  s.sp_y = (float*)dalloc(s, sizeof(float) * N);
  s.sp_x = (float*)dalloc(s, sizeof(float) * (size_t)s.dh * N);
  HIPCHK(hipMemsetAsync(s.sp_y, 0, sizeof(float) * N, s.stream));
  HIPCHK(hipMemsetAsync(s.sp_x, 0, sizeof(float) * (size_t)s.dh * N, s.stream));
  int32_t* cnt = (int32_t*)dalloc(s, sizeof(int32_t) * N);
  HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * N, s.stream));
  HIPCHK(launch_rev_count(s, cnt));
  s.rev_ptr = (int64_t*)dalloc(s, sizeof(int64_t) * (N + 1));
  const int64_t plen = scan_scratch_len((int64_t)N);
  int64_t* part = (int64_t*)dalloc(s, sizeof(int64_t) * (size_t)plen);
  HIPCHK(launch_scan_rows(s, cnt, (int64_t)N, s.rev_ptr, part, plen));
  HIPCHK(hipMemcpyAsync(&s.n_rev, s.rev_ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  dfree(s, part);
  dfree(s, cnt);
  s.rev = (uint64_t*)dalloc(s, sizeof(uint64_t) * (size_t)std::max<int64_t>(s.n_rev, 1));
  unsigned long long* fill = (unsigned long long*)dalloc(s, sizeof(unsigned long long) * N);
  HIPCHK(hipMemcpyAsync(fill, s.rev_ptr, sizeof(int64_t) * N, hipMemcpyDeviceToDevice, s.stream));
  HIPCHK(launch_rev_fill(s, fill));
  HIPCHK(hipStreamSynchronize(s.stream));
  dfree(s, fill);
  // each target's words sorted by source, in chunks of at most 2^27 words
  std::vector<int64_t> h_ptr(N + 1);
  HIPCHK(hipMemcpy(h_ptr.data(), s.rev_ptr, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost));
  const int64_t chunk = std::max<int64_t>(std::min<int64_t>(s.n_rev, (int64_t)1 << 27), 1);
  const int32_t max_segs = 1 << 21;
  size_t temp_bytes = 0;
  HIPCHK(sort_rev_temp_bytes(chunk, max_segs, &temp_bytes));
  uint64_t* alt = (uint64_t*)dalloc(s, sizeof(uint64_t) * (size_t)chunk);
  int32_t* off = (int32_t*)dalloc(s, sizeof(int32_t) * ((size_t)max_segs + 1));
  void* temp = dalloc(s, std::max<size_t>(temp_bytes, 1));
  HIPCHK(sort_rev(s, chunk, max_segs, alt, off, temp, temp_bytes, h_ptr));
  HIPCHK(hipStreamSynchronize(s.stream));
  dfree(s, temp);
  dfree(s, off);
  dfree(s, alt);
}

// Train mode: float32 master weights (initially the int16 weights), their int32 efficacies,
// the adjoint buffers, trajectory recording for one checkpoint segment, checkpoint 0.
void setup_train(sim& s) {
  // the stored canonical permutation keeps each record's offset in its row in 16 bits
  if ((int64_t)s.max_nn * s.npc >= 0xffff)
    throw Fail{DPSNN_EINVAL, "train mode needs rows of fewer than 65535 candidate synapses"};
  const size_t sp = (size_t)s.n_syn_padded + 4;
  const size_t N = (size_t)s.n_neurons;
  // the train-mode step kernel addresses 16-byte pieces from the store's start in 32 bits
  if ((s.n_syn_padded + 4) / 4 >= ((int64_t)1 << 32))
    throw Fail{DPSNN_EINVAL, "train mode needs a store of fewer than 2^34 synapse records"};
  s.wf32 = (float*)dalloc(s, sizeof(float) * sp);
  s.wfx = (int32_t*)dalloc(s, sizeof(int32_t) * sp);
  s.gw = (float*)dalloc(s, sizeof(float) * sp);
  s.dlyw = (uint8_t*)dalloc(s, sp / 4 + 1);
  HIPCHK(hipMemsetAsync(s.dlyw, 0, sp / 4 + 1, s.stream));
  HIPCHK(launch_fill_dly(s));
  HIPCHK(hipMemsetAsync(s.wf32, 0, sizeof(float) * sp, s.stream));
  HIPCHK(hipMemsetAsync(s.wfx, 0, sizeof(int32_t) * sp, s.stream));
  HIPCHK(launch_weights_from_records(s));
  HIPCHK(launch_quantise(s));
  // the canonical order of the weights as a stored permutation (2 B per record), so that the
  // weight and gradient exchanges of every iteration are plain gathers and scatters
  uint16_t* rel = (uint16_t*)dalloc(s, sizeof(uint16_t) * sp);
  HIPCHK(hipMemsetAsync(rel, 0xff, sizeof(uint16_t) * sp, s.stream));
  HIPCHK(launch_canon_perm(s, rel));
  s.canon_rel = rel;
  s.nu_ring = (float*)dalloc(s, sizeof(float) * (size_t)s.dh * N);
  s.adj_gsum = (float*)dalloc(s, sizeof(float) * N);
  s.adj_lam = (float*)dalloc(s, sizeof(float) * N);
  s.adj_mu = (float*)dalloc(s, sizeof(float) * N);
  s.adj_part = (double*)dalloc(s, sizeof(double) * 2 * N);
  s.adj_out = (double*)dalloc(s, sizeof(double) * 2);
  s.loss_rates = (float*)dalloc(s, sizeof(float) * (size_t)s.n_cols);
  s.loss_grad = (float*)dalloc(s, sizeof(float) * (size_t)s.n_cols);
  // single-column native tiles: every part of a row holds the synapses into one column, and
  // the reverse gather can run by target column with that column's future nu in LDS
  if (s.native_tx == 1 && s.native_ty == 1 &&
      adjoint_col_fits(s.npc, s.cfg.d_min, s.cfg.d_max)) {
    std::vector<int32_t> pfirst((size_t)s.n_cols + 1, 0), inp((size_t)s.n_cols * kMaxNbr * 4, -1),
        own((size_t)s.n_cols, -1);
    for (int32_t g = 0; g < s.n_cols; ++g) pfirst[g + 1] = pfirst[g] + s.h_np[g];
    for (int32_t tc = 0; tc < s.n_cols; ++tc)
      for (int i = 0; i < s.h_nn[tc]; ++i) {
        const int32_t src = s.h_nbr[(size_t)tc * kMaxNbr + i];
        int r = 0;
        while (r < s.h_nn[src] && s.h_nbr[(size_t)src * kMaxNbr + r] != tc) ++r;
        if (r == s.h_nn[src]) throw Fail{DPSNN_EINVAL, "column neighbourhoods are not symmetric"};
        int32_t* e = &inp[((size_t)tc * kMaxNbr + i) * 4];
        e[0] = src;
        e[1] = pfirst[src] + s.h_part[(size_t)src * kMaxNbr + r];
        e[2] = pfirst[src];
        e[3] = s.h_np[src];
        if (src == tc) own[tc] = i;
      }
    for (int32_t tc = 0; tc < s.n_cols; ++tc)
      if (own[tc] < 0) throw Fail{DPSNN_EINVAL, "a column is not among its own neighbours"};
    s.in_part = upload(s, inp);
    s.in_own = upload(s, own);
    HIPCHK(prepare_adjoint_kernels());
    s.adj_psum = (float*)dalloc(s, sizeof(float) * (size_t)s.n_idx);
    HIPCHK(hipMemsetAsync(s.adj_psum, 0, sizeof(float) * (size_t)s.n_idx, s.stream));
    s.adj_hsum = (float*)dalloc(s, sizeof(float) * kAdjWindow * (size_t)s.n_idx);
    HIPCHK(hipMemsetAsync(s.adj_hsum, 0, sizeof(float) * kAdjWindow * (size_t)s.n_idx, s.stream));
  }
  s.rec_steps = s.cfg.ckpt_every;
  const size_t rn = (size_t)s.rec_steps * N;
  s.rec_vprev = (float*)dalloc(s, sizeof(float) * rn);
  s.rec_caprev = (float*)dalloc(s, sizeof(float) * rn);
  s.rec_vt = (float*)dalloc(s, sizeof(float) * rn);
  s.rec_flags = (uint8_t*)dalloc(s, rn);
  save_into_ckpt(s, 0);
  s.ckpts[0].epoch = s.epoch;
}

int finish(sim* s, const Fail& f) {
  if (s) s->err = f.msg;
  return f.code;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// sim_create, or with `sizes` set the size query: everything up to the generator's count
// pass, then the region sizes, and the simulation is released again.
int create_impl(const sim_config_t* cfg, const sim_buffers_t* bufs, void* hip_stream,
                sim_t** out, sim_sizes_t* sizes) {
  if (out) *out = nullptr;
  sim* s = nullptr;
  try {
    if (!out && !sizes) throw Fail{DPSNN_EINVAL, "out is NULL"};
    validate(cfg);
    HIPCHK(prepare_step_kernels());
    s = new sim();
    s->cfg = *cfg;
    s->nets.assign(cfg->nets, cfg->nets + cfg->n_nets);
    s->cfg.nets = s->nets.data();
    s->stream = (hipStream_t)hip_stream;
    HIPCHK(hipGetDevice(&s->device));
    s->n_nets = cfg->n_nets;
    s->npc = cfg->npc;
    s->nd = cfg->d_max - cfg->d_min + 1;
    s->dh = cfg->d_max + 1;
    s->idxw = (8 + 2 * (s->nd + 2) + 15) & ~15;
    s->delivery = cfg->delivery == DPSNN_DELIVERY_PUSH ? DPSNN_DELIVERY_PUSH : DPSNN_DELIVERY_ARRIVAL;
    s->block = cfg->block ? cfg->block : default_block(s->delivery);
    set_constants(*s);
    build_tables(*s);
    choose_native(*s, cfg->tile_x, cfg->tile_y);
    build_parts(*s, s->native_tx, s->native_ty);
    build_tiles(*s, s->native_tx, s->native_ty);
    if (sizes) {
      int64_t* part = nullptr;
      int64_t plen = 0;
      const int64_t total = count_records(*s, &part, &plen);
      size_t need[4];
      region_sizes(*s, total, need);
      sizes->n_neurons = s->n_neurons;
      sizes->n_records = total;
      sizes->synapse_bytes = need[kRegSyn];
      sizes->index_bytes = need[kRegIndex];
      sizes->state_bytes = need[kRegState];
      sizes->history_bytes = need[kRegHist];
      sizes->state_v_offset = 0;
      sizes->state_ca_offset = align256(sizeof(float) * (size_t)s->n_neurons);
      sizes->state_ref_offset = 2 * align256(sizeof(float) * (size_t)s->n_neurons);
      sim_destroy(s);
      return DPSNN_OK;
    }
    if (bufs) {
      void* const base[4] = {bufs->synapses, bufs->index, bufs->state, bufs->history};
      const uint64_t cap[4] = {bufs->synapse_bytes, bufs->index_bytes, bufs->state_bytes,
                               bufs->history_bytes};
      for (int r = 0; r < 4; ++r) {
        if (!base[r]) continue;
        if ((uintptr_t)base[r] % 256 != 0)
          throw Fail{DPSNN_EINVAL, std::string("the caller's ") + kRegionName[r] +
                                       " buffer is not 256-byte aligned"};
        s->region_base[r] = (unsigned char*)base[r];
        s->region_cap[r] = (size_t)cap[r];
        s->caller_bytes += (size_t)cap[r];
      }
    }
    generate(*s);
    const size_t N = (size_t)s->n_neurons;
    s->v = (float*)carve(*s, kRegState, sizeof(float) * N);
    s->ca = (float*)carve(*s, kRegState, sizeof(float) * N);
    s->ref = (uint8_t*)carve(*s, kRegState, N);
    if (s->model == kModelLifNa) s->na = (float*)dalloc(*s, sizeof(float) * N);
    s->hist_cnt = (int32_t*)carve(*s, kRegHist, sizeof(int32_t) * (size_t)s->dh * s->n_cols);
    s->hist_ids = (uint16_t*)carve(*s, kRegHist, sizeof(uint16_t) * (size_t)s->dh * s->n_cols * s->npc);
    s->hist_st = (uint64_t*)carve(*s, kRegHist, sizeof(uint64_t) * (size_t)s->dh * s->n_parts * s->npc);
    s->hist_go = (uint16_t*)carve(*s, kRegHist, sizeof(uint16_t) * (size_t)s->dh * s->n_parts * (s->nd + 1) * s->npc);
    s->net_cnt = (unsigned long long*)dalloc(*s, sizeof(unsigned long long) * kCounters * (size_t)s->n_nets);
    s->flags = (int32_t*)dalloc(*s, sizeof(int32_t) * 4);
    s->d_now = (int64_t*)dalloc(*s, sizeof(int64_t));
    s->d_digest = (uint64_t*)dalloc(*s, sizeof(uint64_t));
    s->col_spk = (unsigned long long*)dalloc(*s, sizeof(unsigned long long) * (size_t)s->n_cols);
    s->d_gath = (int64_t*)dalloc(*s, sizeof(int64_t));
    s->d_gdone = (uint32_t*)dalloc(*s, sizeof(uint32_t) * 2);
    HIPCHK(hipMemsetAsync(s->d_gdone, 0, sizeof(uint32_t) * 2, s->stream));
    set_gather(*s, 0);
    HIPCHK(hipMemsetAsync(s->col_spk, 0, sizeof(unsigned long long) * (size_t)s->n_cols, s->stream));
    HIPCHK(hipMemsetAsync(s->hist_cnt, 0, sizeof(int32_t) * (size_t)s->dh * s->n_cols, s->stream));
    HIPCHK(hipMemsetAsync(s->net_cnt, 0, sizeof(unsigned long long) * kCounters * (size_t)s->n_nets, s->stream));
    HIPCHK(hipMemsetAsync(s->flags, 0, sizeof(int32_t) * 4, s->stream));
    HIPCHK(launch_init_state(*s));
    if (s->delivery == DPSNN_DELIVERY_PUSH) ensure_ring(*s);
    if (cfg->record_steps > 0) {
      s->ras_off = (int64_t*)dalloc(*s, sizeof(int64_t) * (size_t)(cfg->record_steps + 1));
      s->ras_ids = (int32_t*)dalloc(*s, sizeof(int32_t) * (size_t)std::max<int64_t>(cfg->raster_capacity, 1));
      s->ras_colofs = (int64_t*)dalloc(*s, sizeof(int64_t) * (size_t)s->n_cols);
      HIPCHK(hipMemsetAsync(s->ras_off, 0, sizeof(int64_t) * (size_t)(cfg->record_steps + 1), s->stream));
    }
    s->snaps.resize(64);
    if (cfg->train_mode) setup_train(*s);
    if (cfg->stdp) setup_stdp(*s);
    HIPCHK(hipStreamSynchronize(s->stream));
    *out = s;
    return DPSNN_OK;
  } catch (const Fail& f) {
    g_create_error = f.msg;
    if (s) sim_destroy(s);
    return f.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    if (s) sim_destroy(s);
    return DPSNN_ENOMEM;
  }
}

}  // namespace

extern "C" {

int sim_query_sizes(const sim_config_t* cfg, sim_sizes_t* sizes) {
  if (!sizes) {
    g_create_error = "sizes is NULL";
    return DPSNN_EINVAL;
  }
  return create_impl(cfg, nullptr, nullptr, nullptr, sizes);
}

int sim_create(const sim_config_t* cfg, const sim_buffers_t* bufs, void* hip_stream, sim_t** out) {
  return create_impl(cfg, bufs, hip_stream, out, nullptr);
}

void sim_destroy(sim_t* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  for (DevBuf& b : s->bufs) (void)hipFree(b.p);
  for (Snapshot& sn : s->snaps) (void)hipFree(sn.blob.p);
  for (Snapshot& sn : s->ckpts) (void)hipFree(sn.blob.p);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

// One step by direct launches (with HIP events around each kernel when timing is on).
static void direct_step(sim& s, std::vector<std::pair<int, size_t>>& marks, size_t& ev_used) {
  auto mark = [&](int cls) -> hipEvent_t {
    if (ev_used + 2 > s.events.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      s.events.push_back(e);
      HIPCHK(hipEventCreate(&e));
      s.events.push_back(e);
    }
    marks.push_back({cls, ev_used});
    ev_used += 2;
    return s.events[ev_used - 2];
  };
  const int64_t u = s.now;
  if (s.timing) {
    HIPCHK(hipEventRecord(mark(0), s.stream));
    HIPCHK(launch_step(s, u, s.delivery, s.block, 0));
    HIPCHK(hipEventRecord(s.events[marks.back().second + 1], s.stream));
    if (s.delivery == DPSNN_DELIVERY_PUSH) {
      HIPCHK(hipEventRecord(mark(1), s.stream));
      HIPCHK(launch_step(s, u, s.delivery, s.block, 1));
      HIPCHK(hipEventRecord(s.events[marks.back().second + 1], s.stream));
    }
  } else {
    HIPCHK(launch_step(s, u, s.delivery, s.block, -1));
  }
  if (s.ras_off && u < s.cfg.record_steps && !s.recompute) {
    if (s.timing) HIPCHK(hipEventRecord(mark(2), s.stream));
    HIPCHK(launch_raster(s, u));
    if (s.timing) HIPCHK(hipEventRecord(s.events[marks.back().second + 1], s.stream));
  }
  s.now = u + 1;
}

static void drop_graph(sim& s) {
  if (s.graph_exec) (void)hipGraphExecDestroy(s.graph_exec);
  s.graph_exec = nullptr;
  s.graph_key.clear();
}

// A graph of `k` steps whose kernels read their step numbers from s.d_now; it is captured
// on a private stream and replayed on the simulation's stream.  Re-captured when the launch
// configuration, the recording state or the step count changes.
static void run_graph_chunk(sim& s, int32_t k, bool record) {
  const std::string key = std::to_string(k) + "/" + std::to_string(s.delivery) + "/" +
                          std::to_string(s.block) + "/" + std::to_string(s.tile_x) + "x" +
                          std::to_string(s.tile_y) + "/" + (record ? "r" : "-") + "/" +
                          (s.rec_on ? "t" : "-") + "/" +
                          std::to_string(s.gk > 1 ? s.now % s.gk : 0);
  if (!s.graph_exec || key != s.graph_key) {
    drop_graph(s);
    if (!s.cap_stream) HIPCHK(hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking));
    hipStream_t user = s.stream;
    s.stream = s.cap_stream;
    s.graph_mode = true;
    s.graph_base = s.now;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal);
    for (int32_t q = 0; q < k && e == hipSuccess; ++q) {
      e = launch_step(s, q, s.delivery, s.block, -1);
      if (e == hipSuccess && record) e = launch_raster(s, q);
    }
    const hipError_t e2 = hipStreamEndCapture(s.cap_stream, &g);
    s.stream = user;
    s.graph_mode = false;
    HIPCHK(e);
    HIPCHK(e2);
    hipGraphExec_t ex = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e3);
    s.graph_exec = ex;
    s.graph_key = key;
  }
  HIPCHK(launch_set_now(s, s.now));
  HIPCHK(hipGraphLaunch(s.graph_exec, s.stream));
  s.now += k;
}

int sim_step(sim_t* s, int64_t n_steps) {
  if (!s) return DPSNN_EINVAL;
  if (n_steps < 0) { s->err = "n_steps < 0"; return DPSNN_EINVAL; }
  if (s->sticky) { s->err = "simulation is in a failed state"; return DPSNN_ESTATE; }
  // every table the step kernels read must be in place (a missing one is a host error, never
  // a launch)
  if (s->delivery == DPSNN_DELIVERY_ARRIVAL &&
      (!s->tile_order || !s->tile_cinfo || !s->tile_ncols || !s->tile_pinfo || !s->tile_net ||
       !s->tile_base || !s->tile_npairs || !s->tile_slots || !s->tile_work || !s->hist_st ||
       !s->hist_go || !s->d_gath || !s->d_gdone || (s->cfg.stdp && (!s->rev || !s->sp_x)))) {
    s->err = "step tables are missing";
    return DPSNN_ESTATE;
  }
  try {
    // with timing on, every kernel launch of the step loop is bracketed by HIP events on
    // the simulation's stream; class 0 = update (fused with delivery in the arrival form),
    // class 1 = push delivery, class 2 = raster recording
    std::vector<std::pair<int, size_t>> marks;  // (class, first event index)
    size_t ev_used = 0;
    int64_t left = n_steps;
    while (left > 0) {
      if (s->wfx) {  // train mode: direct launches, a checkpoint every ckpt_every steps
        // the trajectory of the current segment is recorded on the way, so that the reverse
        // pass need not re-run the last segment when the recording covers all of it
        const int64_t u = s->now, seg = u - u % s->cfg.ckpt_every;
        if (s->rec_base != seg || s->fwd_rec_to != u || s->fwd_rec_epoch != s->epoch) {
          s->rec_base = seg;
          s->fwd_rec_from = u;
          s->fwd_rec_epoch = s->epoch;
        }
        s->fwd_rec_to = -1;
        s->rec_on = true;
        try {
          direct_step(*s, marks, ev_used);
        } catch (...) {
          s->rec_on = false;
          throw;
        }
        s->rec_on = false;
        s->fwd_rec_to = u + 1;
        left -= 1;
        if (s->now % s->cfg.ckpt_every == 0) {
          save_into_ckpt(*s, (size_t)(s->now / s->cfg.ckpt_every));
          s->ckpts[(size_t)(s->now / s->cfg.ckpt_every)].epoch = s->epoch;
        }
        continue;
      }
      const int32_t k = s->graph_steps;
      const bool rec_all = s->ras_off && s->now + k <= s->cfg.record_steps;
      const bool rec_none = !s->ras_off || s->now >= s->cfg.record_steps;
      if (k > 0 && !s->timing && left >= k && (rec_all || rec_none)) {
        run_graph_chunk(*s, k, rec_all);
        left -= k;
      } else {
        direct_step(*s, marks, ev_used);
        left -= 1;
      }
    }
    if (s->timing) {
      for (int c = 0; c < 6; ++c) s->last_ms[c] = 0.0;
      if (!marks.empty()) HIPCHK(hipEventSynchronize(s->events[marks.back().second + 1]));
      for (const auto& m : marks) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, s->events[m.second], s->events[m.second + 1]));
        s->last_ms[m.first] += ms;
        s->last_ms[3 + m.first] += 1.0;
      }
    }
    return DPSNN_OK;
  } catch (const Fail& f) {
    s->sticky = f.code;
    return finish(s, f);
  }
}

int sim_state_digest(sim_t* s, uint64_t* digest) {
  if (!s || !digest) return DPSNN_EINVAL;
  try {
    HIPCHK(launch_digest(*s, s->d_digest));
    HIPCHK(hipMemcpyAsync(digest, s->d_digest, sizeof(uint64_t), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_sync(sim_t* s) {
  if (!s) return DPSNN_EINVAL;
  try {
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->ras_off) {
      int32_t fl = 0;
      HIPCHK(hipMemcpy(&fl, s->flags, sizeof(int32_t), hipMemcpyDeviceToHost));
      if (fl) { s->err = "raster capacity exceeded"; return DPSNN_ETRUNC; }
    }
    if (s->sticky) return DPSNN_ESTATE;
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_read_spikes(sim_t* s, int32_t net, int64_t t0, int64_t t1, int64_t* step_offsets,
                    int32_t* ids, int64_t ids_cap, int64_t* n_ids) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (net < 0 || net >= s->n_nets) throw Fail{DPSNN_EINVAL, "net out of range"};
    if (!s->ras_off) throw Fail{DPSNN_ESTATE, "spike recording is off"};
    const int64_t lim = std::min<int64_t>(s->now, s->cfg.record_steps);
    if (t0 < 0 || t1 < t0 || t1 > lim) throw Fail{DPSNN_EINVAL, "steps outside the recorded window"};
    if (!step_offsets || !n_ids) throw Fail{DPSNN_EINVAL, "NULL output"};
    int rc = sim_sync(s);
    if (rc == DPSNN_ETRUNC) return rc;
    std::vector<int64_t> off((size_t)(t1 - t0 + 1));
    HIPCHK(hipMemcpy(off.data(), s->ras_off + t0, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost));
    if (s->n_nets == 1) {
      // one network holds every id: the recorded rows are the answer as they stand, copied
      // once into the caller's buffer (and not at all for a size query)
      const int64_t cnt = off.back() - off.front();
      for (int64_t t = t0; t <= t1; ++t) step_offsets[t - t0] = off[t - t0] - off.front();
      *n_ids = cnt;
      const int64_t n = ids ? std::min(cnt, ids_cap) : 0;
      if (n > 0)
        HIPCHK(hipMemcpy(ids, s->ras_ids + off.front(), sizeof(int32_t) * (size_t)n,
                         hipMemcpyDeviceToHost));
      if (cnt > ids_cap || (!ids && cnt > 0)) {
        s->err = "ids buffer too small";
        return DPSNN_ETRUNC;
      }
      return DPSNN_OK;
    }
    // several networks: the per-step ranges of this network's ids are found on the device
    // and only those ids cross to the host
    const int32_t lo = s->net_col0[net] * s->npc, hi = s->net_col0[net + 1] * s->npc;
    const int64_t ns = t1 - t0;
    struct Scratch {
      void* p = nullptr;
      ~Scratch() { if (p) (void)hipFree(p); }
    } bnd, take;
    std::vector<int64_t> hb((size_t)(2 * ns));
    if (ns > 0) {
      if (hipMalloc(&bnd.p, sizeof(int64_t) * 3 * (size_t)ns) != hipSuccess) {
        (void)hipGetLastError();
        throw Fail{DPSNN_ENOMEM, "raster read scratch allocation failed"};
      }
      HIPCHK(launch_raster_bounds(*s, t0, ns, lo, hi, (int64_t*)bnd.p));
      HIPCHK(hipMemcpyAsync(hb.data(), bnd.p, sizeof(int64_t) * hb.size(), hipMemcpyDeviceToHost,
                            s->stream));
      HIPCHK(hipStreamSynchronize(s->stream));
    }
    int64_t cnt = 0;
    for (int64_t i = 0; i < ns; ++i) {
      step_offsets[i] = cnt;
      cnt += hb[(size_t)(2 * i + 1)] - hb[(size_t)(2 * i)];
    }
    step_offsets[ns] = cnt;
    *n_ids = cnt;
    const int64_t n = ids ? std::min(cnt, ids_cap) : 0;
    if (n > 0) {
      int64_t* doff = (int64_t*)bnd.p + 2 * ns;
      if (hipMalloc(&take.p, sizeof(int32_t) * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        throw Fail{DPSNN_ENOMEM, "raster read scratch allocation failed"};
      }
      HIPCHK(hipMemcpyAsync(doff, step_offsets, sizeof(int64_t) * (size_t)ns,
                            hipMemcpyHostToDevice, s->stream));
      HIPCHK(launch_raster_take(*s, ns, (const int64_t*)bnd.p, doff, lo, n, (int32_t*)take.p));
      HIPCHK(hipMemcpyAsync(ids, take.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                            s->stream));
      HIPCHK(hipStreamSynchronize(s->stream));
    }
    if (cnt > ids_cap || (!ids && cnt > 0)) {
      s->err = "ids buffer too small";
      return DPSNN_ETRUNC;
    }
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

const char* sim_last_error(const sim_t* s) {
  return s ? s->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

namespace dpsnn {
void set_create_error(const std::string& msg) { g_create_error = msg; }
}  // namespace dpsnn

extern "C" {

int sim_get_info(const sim_t* s, sim_info_t* info) {
  if (!s || !info) return DPSNN_EINVAL;
  info->n_nets = s->n_nets;
  info->n_cols = s->n_cols;
  info->n_neurons = s->n_neurons;
  info->n_synapses = s->n_syn;
  info->ring_slots = s->dh;
  info->device_bytes = (int64_t)s->device_bytes;
  info->caller_bytes = (int64_t)s->caller_bytes;
  return DPSNN_OK;
}

int64_t sim_now(const sim_t* s) { return s ? s->now : -1; }

int sim_get_stats(sim_t* s, int32_t net, sim_stats_t* st) {
  if (!s || !st) return DPSNN_EINVAL;
  try {
    if (net < 0 || net >= s->n_nets) throw Fail{DPSNN_EINVAL, "net out of range"};
    HIPCHK(hipStreamSynchronize(s->stream));
    unsigned long long c[kCounters];
    HIPCHK(hipMemcpy(c, s->net_cnt + kCounters * net, sizeof(c), hipMemcpyDeviceToHost));
    st->steps = s->now;
    st->spikes = (int64_t)c[0];
    st->events_recurrent = (int64_t)c[1];
    st->events_external = (int64_t)c[2];
    st->synapses_streamed = (int64_t)c[3];
    st->synapses_delivered = (int64_t)c[4];
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_read_state(sim_t* s, int32_t net, float* v, float* ca, uint8_t* ref, int32_t* pend,
                   float* na) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (net < 0 || net >= s->n_nets) throw Fail{DPSNN_EINVAL, "net out of range"};
    HIPCHK(hipStreamSynchronize(s->stream));
    const int32_t g0 = s->net_col0[net], g1 = s->net_col0[net + 1];
    const int64_t n0 = (int64_t)g0 * s->npc;
    const size_t nn = (size_t)(g1 - g0) * s->npc;
    if (v) HIPCHK(hipMemcpy(v, s->v + n0, sizeof(float) * nn, hipMemcpyDeviceToHost));
    if (ca) HIPCHK(hipMemcpy(ca, s->ca + n0, sizeof(float) * nn, hipMemcpyDeviceToHost));
    if (ref) HIPCHK(hipMemcpy(ref, s->ref + n0, nn, hipMemcpyDeviceToHost));
    if (na) {
      if (s->na) HIPCHK(hipMemcpy(na, s->na + n0, sizeof(float) * nn, hipMemcpyDeviceToHost));
      else memset(na, 0, sizeof(float) * nn);
    }
    if (pend) {
      if (s->delivery == DPSNN_DELIVERY_PUSH) {
        for (int q = 0; q < s->dh; ++q) {
          const int64_t slot = (s->now + q) % s->dh;
          HIPCHK(hipMemcpy(pend + q * nn, s->ring + slot * s->n_neurons + n0, sizeof(int32_t) * nn,
                           hipMemcpyDeviceToHost));
        }
      } else {
        int32_t* tmp = (int32_t*)dalloc(*s, sizeof(int32_t) * (size_t)s->dh * nn);
        HIPCHK(hipMemsetAsync(tmp, 0, sizeof(int32_t) * (size_t)s->dh * nn, s->stream));
        HIPCHK(launch_pend_view(*s, tmp, g0, g1));
        HIPCHK(hipStreamSynchronize(s->stream));
        HIPCHK(hipMemcpy(pend, tmp, sizeof(int32_t) * (size_t)s->dh * nn, hipMemcpyDeviceToHost));
        dfree(*s, tmp);
      }
    }
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_read_synapses(sim_t* s, int32_t net, int64_t i0, int64_t i1, int64_t* row_ptr,
                      int32_t* tgt, uint8_t* dly, int16_t* wq, int64_t cap) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (net < 0 || net >= s->n_nets) throw Fail{DPSNN_EINVAL, "net out of range"};
    const int64_t nloc = (int64_t)(s->net_col0[net + 1] - s->net_col0[net]) * s->npc;
    if (i0 < 0 || i1 < i0 || i1 > nloc || !row_ptr) throw Fail{DPSNN_EINVAL, "bad row range"};
    HIPCHK(hipStreamSynchronize(s->stream));
    const int64_t g0 = (int64_t)s->net_col0[net] * s->npc + i0;
    const size_t nr = (size_t)(i1 - i0);
    std::vector<int32_t> deg(nr);
    if (nr) HIPCHK(hipMemcpy(deg.data(), s->deg + g0, sizeof(int32_t) * nr, hipMemcpyDeviceToHost));
    row_ptr[0] = 0;
    for (size_t q = 0; q < nr; ++q) row_ptr[q + 1] = row_ptr[q] + deg[q];
    const int64_t total = row_ptr[nr];
    if (total > cap) { s->err = "synapse buffers too small"; return DPSNN_ETRUNC; }
    if (total == 0) return DPSNN_OK;
    if (!tgt || !dly || !wq) throw Fail{DPSNN_EINVAL, "NULL output"};
    // export the padded rows, then drop the padding (delay 0) on the host
    // padded row lengths: the rows of one column follow each other, the last ends at the
    // column's end (columns are stored in folded row order)
    std::vector<int64_t> rb(nr + 1);
    HIPCHK(hipMemcpy(rb.data(), s->row_base + g0, sizeof(int64_t) * rb.size(), hipMemcpyDeviceToHost));
    std::vector<int64_t> poff(nr + 1, 0);
    for (size_t q = 0; q < nr; ++q) {
      const int64_t i = g0 + (int64_t)q;
      const int64_t end = (i + 1) % s->npc == 0 ? s->h_colend[(size_t)(i / s->npc)] : rb[q + 1];
      poff[q + 1] = poff[q] + (end - rb[q]);
    }
    const int64_t ptotal = poff[nr];
    int32_t* dt = (int32_t*)dalloc(*s, sizeof(int32_t) * (size_t)ptotal);
    uint8_t* dd = (uint8_t*)dalloc(*s, (size_t)ptotal);
    int16_t* dw = (int16_t*)dalloc(*s, sizeof(int16_t) * (size_t)ptotal);
    int64_t* doff = (int64_t*)dalloc(*s, sizeof(int64_t) * poff.size());
    HIPCHK(hipMemcpy(doff, poff.data(), sizeof(int64_t) * poff.size(), hipMemcpyHostToDevice));
    HIPCHK(launch_export_rows(*s, net, g0, g0 + (int64_t)nr, dt, dd, dw, doff));
    HIPCHK(hipStreamSynchronize(s->stream));
    std::vector<int32_t> ht((size_t)ptotal);
    std::vector<uint8_t> hd((size_t)ptotal);
    std::vector<int16_t> hw((size_t)ptotal);
    HIPCHK(hipMemcpy(ht.data(), dt, sizeof(int32_t) * (size_t)ptotal, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hd.data(), dd, (size_t)ptotal, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hw.data(), dw, sizeof(int16_t) * (size_t)ptotal, hipMemcpyDeviceToHost));
    dfree(*s, doff);
    dfree(*s, dw);
    dfree(*s, dd);
    dfree(*s, dt);
    // drop the padding and sort each row by (delay, target): the canonical order
    int64_t o = 0;
    std::vector<std::pair<uint64_t, int16_t>> row;
    for (size_t q = 0; q < nr; ++q) {
      row.clear();
      for (int64_t e = poff[q]; e < poff[q + 1]; ++e)
        if (hd[(size_t)e] != 0)
          row.push_back({((uint64_t)hd[(size_t)e] << 32) | (uint32_t)ht[(size_t)e], hw[(size_t)e]});
      std::sort(row.begin(), row.end(),
                [](const std::pair<uint64_t, int16_t>& x, const std::pair<uint64_t, int16_t>& y) {
                  return x.first < y.first;
                });
      if (o + (int64_t)row.size() > total) throw Fail{DPSNN_EHIP, "synapse export overflow"};
      for (const auto& r : row) {
        tgt[o] = (int32_t)(uint32_t)(r.first & 0xffffffffu);
        dly[o] = (uint8_t)(r.first >> 32);
        wq[o] = r.second;
        ++o;
      }
    }
    if (o != total) throw Fail{DPSNN_EHIP, "synapse export is inconsistent with the out-degrees"};
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

}  // extern "C"

namespace {

void save_into(sim& s, Snapshot& sn) {
  size_t parts[kSnapParts];
  void* srcs[kSnapParts];
  snapshot_parts(s, parts, srcs);
  size_t total = 0;
  for (size_t p : parts) total += (p + 255) & ~(size_t)255;
  if (sn.blob.bytes < total) {
    (void)hipFree(sn.blob.p);
    sn.blob.p = nullptr;
    if (hipMalloc(&sn.blob.p, total) != hipSuccess) {
      (void)hipGetLastError();
      sn.blob.bytes = 0;
      throw Fail{DPSNN_ENOMEM, "snapshot allocation failed"};
    }
    sn.blob.bytes = total;
  }
  size_t off = 0;
  for (int q = 0; q < kSnapParts; ++q) {
    if (parts[q])
      HIPCHK(hipMemcpyAsync((char*)sn.blob.p + off, srcs[q], parts[q], hipMemcpyDeviceToDevice, s.stream));
    off += (parts[q] + 255) & ~(size_t)255;
  }
  sn.valid = true;
  sn.now = s.now;
}

void restore_from(sim& s, const Snapshot& sn) {
  if (!sn.valid) throw Fail{DPSNN_ESTATE, "no snapshot in slot"};
  size_t parts[kSnapParts];
  void* dsts[kSnapParts];
  snapshot_parts(s, parts, dsts);
  size_t total = 0;
  for (size_t p : parts) total += (p + 255) & ~(size_t)255;
  if (total > sn.blob.bytes) throw Fail{DPSNN_ESTATE, "snapshot was taken with a different layout"};
  size_t off = 0;
  for (int q = 0; q < kSnapParts; ++q) {
    if (parts[q])
      HIPCHK(hipMemcpyAsync(dsts[q], (char*)sn.blob.p + off, parts[q], hipMemcpyDeviceToDevice, s.stream));
    off += (parts[q] + 255) & ~(size_t)255;
  }
  s.now = sn.now;
  // the history entries and the push ring are functions of the spike history: rebuild them
  HIPCHK(launch_fill_entries(s));
  invalidate_gather(s);
  if (s.delivery == DPSNN_DELIVERY_PUSH) ring_from_history(s);
}

// Train mode: a state from another recorded window (or a change of weights or parameters
// after step 0) breaks the window; sim_backward then refuses until sim_rewind.
void break_window(sim& s) {
  ++s.epoch;
  if (s.now == 0 && !s.ckpts.empty()) s.ckpts[0].epoch = s.epoch;
}

void save_into_ckpt(sim& s, size_t m) {
  if (s.ckpts.size() <= m) s.ckpts.resize(m + 1);
  save_into(s, s.ckpts[m]);
}

}  // namespace

extern "C" {

int sim_save(sim_t* s, int32_t slot) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (slot < 0 || slot >= 64) throw Fail{DPSNN_EINVAL, "slot out of range"};
    save_into(*s, s->snaps[slot]);
    s->snaps[slot].epoch = s->epoch;
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_restore(sim_t* s, int32_t slot) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (slot < 0 || slot >= 64) throw Fail{DPSNN_EINVAL, "slot out of range"};
    const bool same_window = s->snaps[slot].epoch == s->epoch;
    restore_from(*s, s->snaps[slot]);
    if (s->wfx && !same_window) break_window(*s);
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_set_params(sim_t* s, double tau_m, double g_ahp) {
  if (!s) return DPSNN_EINVAL;
  if (!(tau_m > 0)) { s->err = "tau_m must be positive"; return DPSNN_EINVAL; }
  s->cfg.tau_m = tau_m;
  s->cfg.g_ahp = g_ahp;
  set_constants(*s);
  // the constants reach the kernels by value: a captured step graph holds the old ones
  drop_graph(*s);
  if (s->wfx) break_window(*s);
  return DPSNN_OK;
}

int sim_get_launch(const sim_t* s, sim_launch_t* l) {
  if (!s || !l) return DPSNN_EINVAL;
  l->delivery = s->delivery;
  l->block = s->block;
  l->tile_x = s->tile_x;
  l->tile_y = s->tile_y;
  l->graph_steps = s->graph_steps;
  l->gather_steps = s->gk;
  return DPSNN_OK;
}

int sim_set_launch(sim_t* s, const sim_launch_t* l) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (!l) throw Fail{DPSNN_EINVAL, "launch is NULL"};
    const int32_t block = l->block;
    if (!(block == 64 || block == 128 || block == 256 || block == 512 || block == 1024))
      throw Fail{DPSNN_EINVAL, "block must be 64, 128, 256, 512 or 1024"};
    if (l->delivery != DPSNN_DELIVERY_ARRIVAL && l->delivery != DPSNN_DELIVERY_PUSH)
      throw Fail{DPSNN_EINVAL, "delivery must be ARRIVAL or PUSH"};
    if (l->graph_steps < 0 || l->graph_steps > 4096)
      throw Fail{DPSNN_EINVAL, "graph_steps must be in [0, 4096]"};
    if (l->gather_steps < 0 || l->gather_steps > kMaxGather)
      throw Fail{DPSNN_EINVAL, "gather_steps must be in [0, 8]"};
    if (s->cfg.stdp && (l->delivery != DPSNN_DELIVERY_ARRIVAL || l->tile_x != s->tile_x ||
                        l->tile_y != s->tile_y || l->gather_steps > 1))
      throw Fail{DPSNN_EINVAL, "with STDP the delivery, the tiling and one step per gather are "
                               "fixed"};
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(*s);
    s->graph_steps = l->graph_steps;
    if (l->tile_x != s->tile_x || l->tile_y != s->tile_y) {
      s->gk = 1;
      build_tiles(*s, l->tile_x, l->tile_y);
    }
    if (l->delivery == DPSNN_DELIVERY_PUSH && s->delivery != DPSNN_DELIVERY_PUSH) ring_from_history(*s);
    s->delivery = l->delivery;
    s->block = block;
    set_gather(*s, l->gather_steps);
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_set_timing(sim_t* s, int32_t on) {
  if (!s) return DPSNN_EINVAL;
  s->timing = on != 0;
  return DPSNN_OK;
}

int sim_get_timing(sim_t* s, double* ms, int32_t n) {
  if (!s || !ms) return DPSNN_EINVAL;
  for (int q = 0; q < n && q < 6; ++q) ms[q] = s->last_ms[q];
  return DPSNN_OK;
}

static void need_train(const sim& s) {
  if (!s.wfx) throw Fail{DPSNN_ESTATE, "not in train mode"};
}

int sim_set_weights(sim_t* s, const float* w) {
  if (!s) return DPSNN_EINVAL;
  try {
    need_train(*s);
    if (!w) throw Fail{DPSNN_EINVAL, "w is NULL"};
    HIPCHK(launch_canon_map(*s, 0, w, s->wf32));
    HIPCHK(launch_quantise(*s));
    invalidate_gather(*s);
    break_window(*s);
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_get_weights(sim_t* s, float* w) {
  if (!s) return DPSNN_EINVAL;
  try {
    need_train(*s);
    if (!w) throw Fail{DPSNN_EINVAL, "w is NULL"};
    HIPCHK(launch_canon_map(*s, 1, s->wf32, w));
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_rewind(sim_t* s) {
  if (!s) return DPSNN_EINVAL;
  try {
    need_train(*s);
    restore_from(*s, s->ckpts[0]);
    ++s->epoch;
    s->ckpts[0].epoch = s->epoch;
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

int sim_column_rates(sim_t* s, float* rates) {
  if (!s) return DPSNN_EINVAL;
  try {
    if (!rates) throw Fail{DPSNN_EINVAL, "rates is NULL"};
    if (s->now == 0) throw Fail{DPSNN_ESTATE, "no steps since step 0"};
    const double scale = 1000.0 / ((double)s->npc * (double)s->now * s->cfg.dt);
    HIPCHK(launch_column_rates(*s, (float)scale, rates));
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

// Reverse pass over the recorded window [0, T): the end state is set aside, then for each
// checkpoint segment from the last to the first the forward is re-run from its checkpoint
// with the trajectory recorded (the last segment only when the forward's own recording does
// not hold all of it), and the adjoint recursion runs backwards through it.  The
// adjoint ring carries nu across segment boundaries.  Finally the end state comes back.
int sim_backward(sim_t* s, const float* target_rates, float* loss, float* grad_w,
                 double* grad_tau_m, double* grad_g_ahp) {
  if (!s) return DPSNN_EINVAL;
  if (s->sticky) { s->err = "simulation is in a failed state"; return DPSNN_ESTATE; }
  try {
    need_train(*s);
    if (!target_rates || !grad_w) throw Fail{DPSNN_EINVAL, "target_rates and grad_w are required"};
    if (s->now == 0) throw Fail{DPSNN_ESTATE, "nothing recorded: no steps since step 0"};
    const double scale = 1000.0 / ((double)s->npc * (double)s->now * s->cfg.dt);
    HIPCHK(launch_column_rates(*s, (float)scale, s->loss_rates));
    HIPCHK(launch_rate_loss(*s, s->loss_rates, target_rates, loss, s->loss_grad));
  } catch (const Fail& f) {
    return finish(s, f);
  }
  return sim_backward_rates(s, s->loss_grad, grad_w, grad_tau_m, grad_g_ahp);
}

int sim_backward_rates(sim_t* s, const float* grad_rates, float* grad_w, double* grad_tau_m,
                       double* grad_g_ahp) {
  if (!s) return DPSNN_EINVAL;
  if (s->sticky) { s->err = "simulation is in a failed state"; return DPSNN_ESTATE; }
  try {
    need_train(*s);
    if (!grad_rates || !grad_w) throw Fail{DPSNN_EINVAL, "grad_rates and grad_w are required"};
    const int64_t T = s->now, K = s->cfg.ckpt_every;
    if (T == 0) throw Fail{DPSNN_ESTATE, "nothing recorded: no steps since step 0"};
    const int64_t M = (T + K - 1) / K;
    if ((int64_t)s->ckpts.size() < M) throw Fail{DPSNN_ESTATE, "recorded window is incomplete; call sim_rewind"};
    for (int64_t m = 0; m < M; ++m)
      if (!s->ckpts[(size_t)m].valid || s->ckpts[(size_t)m].epoch != s->epoch)
        throw Fail{DPSNN_ESTATE, "recorded window was broken by a restore, a weight or a "
                                 "parameter change; call sim_rewind"};
    const size_t N = (size_t)s->n_neurons;
    save_into(*s, s->bwd_end);
    HIPCHK(hipMemsetAsync(s->nu_ring, 0, sizeof(float) * (size_t)s->dh * N, s->stream));
    HIPCHK(hipMemsetAsync(s->adj_lam, 0, sizeof(float) * N, s->stream));
    HIPCHK(hipMemsetAsync(s->adj_mu, 0, sizeof(float) * N, s->stream));
    HIPCHK(hipMemsetAsync(s->adj_part, 0, sizeof(double) * 2 * N, s->stream));
    HIPCHK(hipMemsetAsync(s->gw, 0, sizeof(float) * ((size_t)s->n_syn_padded + 4), s->stream));
    const float scale = (float)(1000.0 / ((double)s->npc * (double)T * s->cfg.dt));
    const bool timing = s->timing;
    s->timing = false;
    std::vector<std::pair<int, size_t>> marks;
    size_t ev_used = 0;
    // the forward's own recording serves the last segment when it covers all of it
    const bool have_last = s->rec_base == (M - 1) * K && s->fwd_rec_from == s->rec_base &&
                           s->fwd_rec_to == T && s->fwd_rec_epoch == s->epoch;
    s->fwd_rec_to = -1;  // the recording buffers are rewritten below
    for (int64_t m = M - 1; m >= 0; --m) {
      const int64_t u0 = m * K, u1 = std::min(T, u0 + K);
      if (!(m == M - 1 && have_last)) {
        restore_from(*s, s->ckpts[(size_t)m]);
        s->rec_on = true;
        s->recompute = true;
        s->rec_base = u0;
        try {
          while (s->now < u1) direct_step(*s, marks, ev_used);
        } catch (...) {
          s->rec_on = false;
          s->recompute = false;
          s->timing = timing;
          throw;
        }
        s->rec_on = false;
        s->recompute = false;
      }
      s->rec_base = u0;
      for (int64_t u = u1 - 1; u >= u0;)
        HIPCHK(launch_adjoint_window(*s, u, u0, grad_rates, scale, (float)s->cfg.surrogate_beta,
                                     &u));
    }
    s->timing = timing;
    HIPCHK(launch_reduce_parts(*s, s->adj_out));
    double out[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(out, s->adj_out, sizeof(out), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(launch_canon_map(*s, 1, s->gw, grad_w));
    restore_from(*s, s->bwd_end);
    HIPCHK(hipStreamSynchronize(s->stream));
    // P_m = exp(-dt / tau_m): dP_m/dtau_m = P_m dt / tau_m^2;  gamma = g_AHP dt
    const double dt = s->cfg.dt, tau = s->cfg.tau_m;
    const double pm = exp(-dt / tau);
    if (grad_tau_m) *grad_tau_m = out[0] * pm * dt / (tau * tau);
    if (grad_g_ahp) *grad_g_ahp = out[1] * dt;
    return DPSNN_OK;
  } catch (const Fail& f) {
    return finish(s, f);
  }
}

}  // extern "C"
