// dpsnn_internal.h -- internal structures and device helpers of libdpsnn (gfx950).
//
// Device data layout (all networks of a simulation concatenated column by column; the
// global neuron index is g*npc + k for global column g and local index k):
//
//   synapse store: rows are stored column by column, the columns of a network in folded
//   row order (grid rows 0, R-1, 1, R-2, 2, ...; inside a row by x; inside a column by
//   neuron), so that the rows of stencil neighbours -- across the torus' wrap included --
//   lie within a few grid rows of each other (row_base[i] gives any row's start).
//   The canonical order of a row is (delay, target); the device keeps each
//   row split into parts, one per target tile of the tiling chosen at creation (the
//   "native" tiling): part p of a source column holds the synapses whose target column
//   lies in the p-th distinct tile touched by the column's stencil (3x3, or up to 7x7 with
//   the Gaussian kernel).  A part is a sequence of groups, one per delay; inside a group
//   the targets come in canonical order.  A synapse's target column is identified by its
//   rank r inside its part: the part's columns, ascending, are part_col[part][0..8] (at
//   most 9 columns per part)
//     idx       idxw bytes per (neuron, part): int64 start of the part, then uint16
//               goff[nd + 1], then the uint16 count of the part's synapses (without the
//               padding); group dd (delay d_min + dd) is [start + goff[dd], start +
//               goff[dd + 1]).  Entry of (column g, neuron k, part p): col_pbase[g] +
//               k * col_np[g] + p.  The parts of one neuron are contiguous (row_base[i])
//     syn       uint32[S' + 4]: k (bits 0-11, target index inside its column) | r (bits
//               12-15, rank in the part) | w_q (bits 16-31, int16 weight at 2^-14 mV).  Every
//               group is padded
//               to a multiple of 4 records with dummies (r = 9, weight 0), so parts and
//               groups start on 16-byte boundaries and are read in whole 16-byte words
//     deg       int32 [N]    out-degree (records without the padding)
//     wfx       int32 [S']   train mode only: rint(w_f32 * 2^16) efficacies
//   column tables (kMaxNbr = 49 entries per column: the 7x7 stencil)
//     col_nbr   int32 [C][49]  distinct stencil columns, ascending, -1 padded
//     col_thr   uint64[C][49]  pair connection threshold from g to col_nbr[g][r]
//     col_part  int32 [C][49]  part of stencil rank r (-1 padded); col_prank the rank of
//                              col_nbr[g][r] inside its part; col_np int32 [C] parts per
//                              column; col_pbase int64 [C+1] first idx entry of the column
//     part_col  int32 [P][9]   the columns of every part by rank (part_srank: their stencil
//                              ranks)
//   tiles (the unit of work of the arrival kernel): up to 4x4 target columns of one network
//     tile_cinfo  int32x4 [tiles][16] per column of the tile: column (-1 padded), index
//                                     within its network, parts, first part index
//     tile_pinfo  int32x2 [tiles][128] every (source column, global part index) with a
//                                     synapse into the tile, -1 padded (one part per source
//                                     in the native tiling; a part may reach several tiles
//                                     otherwise)
//     tile_net    int32 [tiles]       the tile's network
//     tile_base   int64 [tiles]       the first 16-byte piece of the rows of the tile's source
//                                     columns: the tile kernel addresses pieces relative to
//                                     it in 32 bits (a tile's sources lie within a few grid
//                                     rows of columns, far less than 2^32 pieces)
//     tile_slots  uint64[tiles][128]  for each pair and each rank r of its part, the tile
//                                     slot of its target column in bits 5r..5r+4 (31: not
//                                     in the tile or not in the part); bits 45-63 are set
//   spike history (shared by both delivery strategies)
//     hist_cnt  int32 [DH][C]       spikes of column g at step t, in slot t % DH
//     hist_ids  uint16[DH][C][npc]  their local indices, ascending
//     hist_st   uint64 [DH][P][npc] per part (P = parts of all columns, part q of column g
//                                   is col_pfirst[g] + q) and spike position: the start of
//                                   the spiking neuron's part in 16-byte pieces (parts start
//                                   on 16-byte boundaries)
//     hist_go   uint16[DH][P][nd+1][npc]  its group offsets (copied from the row index when
//                                   the neuron spiked, so that the readers of one source
//                                   column's spikes load them contiguously)
//   plasticity (only with stdp on; the store is then written by the step kernels)
//     sp_y      float [N]         postsynaptic trace after the last step
//     sp_x      float [DH][N]     presynaptic trace of step t in slot t % DH
//     rev_ptr   int64 [N+1]       the plastic synapses into each neuron ...
//     rev       uint64 [S+]       ... each as record index | (delay - 1) << 35 | source << 40
//   push-delivery ring (only with DPSNN_DELIVERY_PUSH)
//     ring      int32 [DH][N]       input of step t in slot t % DH
//
// DH = d_max + 1 slots: a step reads slots of steps t-d_max .. t-1 and writes slot t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dpsnn.h"

namespace dpsnn {

constexpr int kMaxNbr = 49;         // distinct columns of a stencil (7x7 at most)
constexpr int kMaxNbr3x3 = 9;       // of the 3x3 stencil
constexpr int kMaxPartCols = 9;     // columns of one part (the 4-bit rank field: 0..8)
constexpr int kMaxNpc = 4096;       // 12-bit target index
constexpr int kMaxDelay = 32;
constexpr int kPoissonEntries = 63;
constexpr int kMaxTileSide = 4;
constexpr int kMaxTileCols = kMaxTileSide * kMaxTileSide;
constexpr int kMaxTilePairs = 128;  // (source column, part) pairs of one tile
constexpr int kMaxParts = 16;       // parts of one source column
constexpr int kNoSlot = 31;
// dummy records carry rank 9, one past the last part rank: the slot words' fields from the
// tenth up read 31, so a dummy decodes as "not in the tile" without clamping its rank
constexpr int kDummyRank = kMaxPartCols;
constexpr uint32_t kDummyRecord = (uint32_t)kDummyRank << 12;  // k 0, rank 9, weight 0
constexpr int kCounters = 8;        // per-network counters (see StepArgs::net_cnt)
constexpr int kAdjWindow = 3;       // reverse steps per window of the column-wise adjoint gather
constexpr size_t kMaxLds = 160 * 1024;
constexpr uint32_t kStreamSyn = 1;  // Philox counter word 3: purpose of the draw
constexpr uint32_t kStreamExt = 2;
constexpr uint32_t kStreamInit = 3;

// record fields
__host__ __device__ __forceinline__ uint32_t rec_k(uint32_t w) { return w & 0xfffu; }
__host__ __device__ __forceinline__ uint32_t rec_rank(uint32_t w) { return (w >> 12) & 0xfu; }
__host__ __device__ __forceinline__ int32_t rec_w32(uint32_t w) { return (((int32_t)w) >> 16) * 4; }
// the weight in its own 2^-14 mV units
__host__ __device__ __forceinline__ int32_t rec_wq(uint32_t w) { return ((int32_t)w) >> 16; }

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products, high halves
// xor-ed with the other counter words and the key, key advanced by the Weyl increments.
// ---------------------------------------------------------------------------------------
struct Rand4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Rand4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Rand4{c0, c1, c2, c3};
}

// Neuron models of the step kernels (a template parameter): LIF with the calcium AHP only,
// LIF with the calcium and sodium AHP variables, Izhikevich RS/FS.
constexpr int kModelLif = 0;
constexpr int kModelLifNa = 1;
constexpr int kModelIzh = 2;

// Neuron constants, rounded once from double on the host.
struct NeuronK {
  float pm;      // exp(-dt / tau_m)
  float pc;      // exp(-dt / tau_ca)
  float gam;     // g_ahp * dt
  float alpha;   // calcium increment
  float theta;
  float vreset;
  int32_t jfx;   // rint(j_ext * 2^16)
  int32_t tref;
  float pna;     // exp(-dt / tau_na)
  float gna;     // g_na * dt
  float alpha_na;  // sodium-variable increment
  float vpeak;   // Izhikevich spike cut-off
  float ia[2], ib[2], ic[2], id[2];  // Izhikevich a, b, c, d: [0] excitatory, [1] inhibitory
};

// Everything the step kernels read or write, by value.
struct StepArgs {
  // sizes
  int32_t npc, nd, d_min, dh, n_cols, idxw;
  int32_t n_exc;               // local index k < n_exc: excitatory
  // step numbers: u = u_arg + *now_dev when now_dev is set (replayable graph steps)
  const int64_t* now_dev;
  // column / network tables
  const int32_t* col_net;
  const int32_t* col_local;   // column index within its network
  const int32_t* col_nbr;
  const int32_t* col_nn;
  const int32_t* col_np;      // parts per column
  const int32_t* col_part;    // [C][9]: part of each neighbour rank
  const int64_t* col_pbase;   // first row-index entry of each column
  const int32_t* col_pfirst;  // first part index of each column
  const int32_t* part_col;    // [P][kMaxPartCols]: column of each rank of each part
  const int32_t* part_srank;  // [P][kMaxPartCols]: its stencil rank in the source column
  int32_t n_parts;
  const int32_t* col_order;   // [grid_cols]: column of workgroup b of per-column kernels
  int32_t grid_cols;
  const uint32_t* net_key;    // [n_nets][2]
  const uint64_t* net_ptab;   // [n_nets][63]
  // tiles
  int32_t* tile_order;        // [grid_tiles]: tile of workgroup b (-1: none)
  int32_t grid_tiles;
  int32_t n_tiles;
  uint32_t* tile_work;        // [n_tiles]: synapse records read at the last gathering step
  int32_t order_by_work;      // reorder tiles by work after each gathering step
  const int4* tile_cinfo;
  const int32_t* tile_ncols;
  const int2* tile_pinfo;
  const int32_t* tile_net;
  const int64_t* tile_base;   // [n_tiles] first piece of the tile's source rows
  const int32_t* tile_npairs;
  const uint64_t* tile_slots;
  // synapses
  const int64_t* row_base;
  const int32_t* deg;
  const uint8_t* idx;
  const uint32_t* syn;
  const int32_t* wfx;         // train mode, else null
  // state
  float* v;
  float* ca;                  // calcium (LIF) or the recovery variable u (Izhikevich)
  float* na;                  // sodium AHP variable (LIF with g_na != 0), else null
  uint8_t* ref;
  int32_t* hist_cnt;
  uint16_t* hist_ids;
  uint64_t* hist_st;
  uint16_t* hist_go;
  // arrival form: steps gathered per window, accumulators of later steps, last gathering
  // step, finished workgroups and next tile of a tile launch
  int32_t gk;
  int32_t* acc_save;          // [gk][N]
  int64_t* gath;
  uint32_t* gdone;
  int32_t* ring;              // push only
  unsigned long long* net_cnt;  // [n_nets][kCounters]: spikes, e_rec, e_ext, synapse records
                                // read, synapses delivered (arrival form)
  unsigned long long* col_spk;  // [n_cols]: spikes per column
  // plasticity (null / unused when off): the store, writable; the postsynaptic trace y and
  // the presynaptic traces x of the last DH steps; the synapses into each neuron
  uint32_t* syn_rw;
  float* sp_y;                // [N] after the last step
  float* sp_x;                // [DH][N], step t in slot t % DH
  const int64_t* rev_ptr;     // [N+1]
  const uint64_t* rev;        // record index (bits 0-34) | delay - 1 (35-39) | source (40-63)
  float sp_pp, sp_pm;         // exp(-dt / tau_plus), exp(-dt / tau_minus)
  float sp_ap, sp_am;         // a_plus, a_minus (mV)
  int32_t sp_qmax;            // rint(w_max * 2^14)
  // train-mode trajectory recording (null when off): [steps][N]
  float* rec_vprev;
  float* rec_caprev;
  float* rec_vt;
  uint8_t* rec_flags;         // bit0 spike, bit1 refractory
  int64_t rec_base;           // first step held by the recording buffers
  NeuronK k;
};

// row-index entry of part p of neuron k of column g
__device__ __forceinline__ const uint8_t* idx_entry(const StepArgs& a, int32_t g, int32_t k,
                                                     int p) {
  return a.idx + (a.col_pbase[g] + (int64_t)k * a.col_np[g] + p) * a.idxw;
}
__device__ __forceinline__ int64_t ent_start(const uint8_t* e) { return *(const int64_t*)e; }
__device__ __forceinline__ const uint16_t* ent_goff(const uint8_t* e) {
  return (const uint16_t*)(e + 8);
}

// Spike-history entries of a spike of neuron k of column g at position pos of slot `slot`:
// for every part, the part's start and group offsets, copied from the row index.
__device__ __forceinline__ void write_entries(const StepArgs& a, int32_t g, int32_t k,
                                              int32_t slot, int32_t pos) {
  const int np = a.col_np[g];
  for (int p = 0; p < np; ++p) {
    const uint8_t* ent = idx_entry(a, g, k, p);
    const int64_t pid = (int64_t)slot * a.n_parts + a.col_pfirst[g] + p;
    a.hist_st[pid * a.npc + pos] = (uint64_t)(ent_start(ent) >> 2);
    const uint16_t* go = ent_goff(ent);
    uint16_t* out = a.hist_go + pid * (int64_t)(a.nd + 1) * a.npc + pos;
    for (int dd = 0; dd <= a.nd; ++dd) out[(int64_t)dd * a.npc] = go[dd];
  }
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Snapshot {
  bool valid = false;
  int64_t now = 0;
  int64_t epoch = 0;  // train mode: recorded window the state belongs to
  DevBuf blob;  // v | ca | ref | hist_cnt | hist_ids | net_cnt | col_spk
};

}  // namespace dpsnn

struct sim {
  sim_config_t cfg;
  std::vector<sim_net_t> nets;
  hipStream_t stream = nullptr;
  int device = 0;                   // HIP device current at creation
  std::string err;
  int sticky = 0;

  // sizes
  int32_t n_nets = 0, n_cols = 0, npc = 0, nd = 0, dh = 0, idxw = 0;
  int64_t n_neurons = 0, n_syn = 0, n_syn_padded = 0;
  std::vector<int32_t> net_col0;    // first global column of each network (n_nets+1)
  std::vector<int64_t> net_syn0;    // first synapse of each network (n_nets+1)
  std::vector<int32_t> h_nbr, h_nn; // host copies of the neighbour tables

  // device memory
  std::vector<dpsnn::DevBuf> bufs;
  size_t device_bytes = 0;
  // caller-owned regions (sim_buffers_t): synapses, index, state, history; base null when
  // the library allocates that region's arrays itself
  unsigned char* region_base[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t region_cap[4] = {0, 0, 0, 0};
  size_t region_used[4] = {0, 0, 0, 0};
  size_t caller_bytes = 0;
  float* loss_rates = nullptr;     // train mode: column rates and dL/dR of the built-in loss
  float* loss_grad = nullptr;
  int32_t *col_net = nullptr, *col_local = nullptr, *col_nbr = nullptr, *col_nn = nullptr;
  int32_t *col_part = nullptr, *col_np = nullptr, *col_prank = nullptr;
  int64_t* col_pbase = nullptr;
  int32_t* col_pfirst = nullptr;
  int32_t *part_col = nullptr, *part_srank = nullptr;
  int32_t n_parts = 0;
  int32_t max_nn = 0;                 // most distinct stencil columns of any column
  std::vector<int32_t> h_part, h_np, h_prank;  // host copies of the part tables
  int64_t n_idx = 0;                  // row-index entries (neuron, part)
  int32_t native_tx = 0, native_ty = 0;  // tiling of the synapse parts
  int32_t* col_order = nullptr;
  int32_t grid_cols = 0;
  uint64_t* col_thr = nullptr;
  uint32_t* net_key = nullptr;
  uint64_t* net_ptab = nullptr;
  int64_t* row_base = nullptr;
  int32_t* deg = nullptr;
  uint8_t* idx = nullptr;
  uint32_t* syn = nullptr;
  int32_t* wfx = nullptr;
  float* wf32 = nullptr;
  float *v = nullptr, *ca = nullptr, *na = nullptr;
  uint8_t* ref = nullptr;
  int32_t model = dpsnn::kModelLif;  // kModel* of the step kernels
  int32_t* hist_cnt = nullptr;
  uint16_t* hist_ids = nullptr;
  uint64_t* hist_st = nullptr;
  uint16_t* hist_go = nullptr;
  int32_t gk = 1;                  // steps gathered per window (arrival form)
  int32_t gather_req = 0;          // requested gather_steps (0: automatic)
  int32_t* acc_save = nullptr;     // [gk][N] accumulators of the later steps of a window
  int64_t* d_gath = nullptr;       // last gathering step, -1 when acc_save is not valid
  uint32_t* d_gdone = nullptr;     // [0] finished workgroups of a tile launch, [1] next tile
  int32_t* ring = nullptr;
  unsigned long long* net_cnt = nullptr;
  // plasticity (cfg.stdp)
  float *sp_y = nullptr, *sp_x = nullptr;
  int64_t* rev_ptr = nullptr;
  uint64_t* rev = nullptr;
  int64_t n_rev = 0;
  // tiles of the current shape
  int32_t tile_x = 0, tile_y = 0, n_tiles = 0, grid_tiles = 0, tile_max_cols = 0;
  int32_t *tile_order = nullptr, *tile_cinfo = nullptr, *tile_ncols = nullptr,
          *tile_pinfo = nullptr, *tile_net = nullptr, *tile_npairs = nullptr;
  uint64_t* tile_slots = nullptr;
  int64_t* tile_base = nullptr;    // [n_tiles] first piece of each tile's source rows
  std::vector<int32_t> h_tile_src;  // source columns of every tile, from h_tile_src_off[t]
  std::vector<int32_t> h_tile_src_off;  // [n_tiles + 1]
  std::vector<int64_t> h_colstart;  // [C] first record of each column's rows (after the count
  std::vector<int64_t> h_colend;    // [C]   pass) and one past its last
  int64_t* col_end = nullptr;       // [C] device copy of h_colend
  uint32_t* tile_work = nullptr;   // [n_tiles] records read per tile at the last gathering step
  int32_t order_by_work = 0;       // more tiles than compute units: order them by work
  // raster
  int64_t* ras_off = nullptr;      // [record_steps+1]
  int32_t* ras_ids = nullptr;      // [raster_capacity], global neuron ids
  int64_t* ras_colofs = nullptr;   // [C] scratch
  int32_t* flags = nullptr;        // [4]: raster overflow
  unsigned long long* col_spk = nullptr;
  // train mode
  float *rec_vprev = nullptr, *rec_caprev = nullptr, *rec_vt = nullptr;
  uint8_t* rec_flags = nullptr;
  int64_t rec_steps = 0;
  int64_t rec_base = 0;
  bool rec_on = false;
  // the train-mode forward records its current checkpoint segment as it steps: steps
  // [fwd_rec_from, fwd_rec_to) of the segment at rec_base, in window epoch fwd_rec_epoch
  int64_t fwd_rec_from = -1, fwd_rec_to = -1, fwd_rec_epoch = -1;
  float* gw = nullptr;             // weight gradient, padded layout
  uint8_t* dlyw = nullptr;         // delay index of each 16-byte word of records
  float* nu_ring = nullptr;        // [dh][N] adjoint of V~ of the last dh steps
  float *adj_gsum = nullptr, *adj_lam = nullptr, *adj_mu = nullptr;
  double* adj_part = nullptr;      // [2][N]
  int32_t* in_part = nullptr;      // [C][9][4] single-column parts: the i-th source column
                                   // of column C, its global part into C, its first part and
                                   // part count (null otherwise)
  int32_t* in_own = nullptr;       // [C] position of C among its own source columns
  float* adj_psum = nullptr;       // [parts][npc] adjoint gather per part (with in_part)
  float* adj_hsum = nullptr;       // [kAdjWindow][parts][npc] its heavy-pass sums per window
  double* adj_out = nullptr;       // [2]
  int64_t* canon_start = nullptr;  // [N+1] first canonical synapse index of each row
  uint16_t* canon_rel = nullptr;   // [S'+4] canonical index of each record minus its row's
                                   // canon_start (0xffff: padding)
  std::vector<dpsnn::Snapshot> ckpts;  // state at steps 0, K, 2K, ... of the recorded window
  dpsnn::Snapshot bwd_end;             // state at the end of the window during sim_backward
  int64_t epoch = 0;               // recorded-window counter (rewind, weight or parameter change)
  bool recompute = false;          // re-running a checkpoint segment: no raster recording

  int64_t now = 0;
  int32_t delivery = DPSNN_DELIVERY_ARRIVAL;
  int32_t block = 256;
  dpsnn::NeuronK nk;
  std::vector<dpsnn::Snapshot> snaps;

  bool timing = false;
  double last_ms[6] = {0, 0, 0, 0, 0, 0};
  std::vector<hipEvent_t> events;

  // replayable step graphs
  int64_t* d_now = nullptr;        // device step base read by graph-launched kernels
  int32_t graph_steps = 0;         // steps per captured graph (0: direct launches)
  bool graph_mode = false;         // true while capturing: kernels read d_now
  int64_t graph_base = 0;          // while capturing: the step the graph's first step stands for
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::string graph_key;
  uint64_t* d_digest = nullptr;
};

namespace dpsnn {

// launchers implemented in the .hip files (host functions)
hipError_t launch_gen_count(const sim& s, int64_t row0, int64_t rows, int32_t* row_len);
hipError_t launch_gen_fill(const sim& s, int64_t row0, int64_t rows);
hipError_t launch_scan_rows(const sim& s, const int32_t* row_len, int64_t n, int64_t* out,
                            int64_t* scratch, int64_t scratch_len);
hipError_t launch_fold_rows(const sim& s, const int64_t* old_start, const int64_t* new_start);
hipError_t launch_init_state(const sim& s);
// part: -1 the whole step, 0 the update (fused with the gather in the arrival form),
// 1 the push delivery
hipError_t launch_step(sim& s, int64_t u, int32_t delivery, int32_t block, int part);
size_t tile_lds_bytes(const sim& s, int32_t kacc);
hipError_t prepare_step_kernels();
bool tile_lds_ok(const sim& s);
hipError_t launch_raster(sim& s, int64_t u);
hipError_t launch_set_now(const sim& s, int64_t now);
hipError_t launch_digest(const sim& s, uint64_t* out);
hipError_t launch_pend_view(const sim& s, int32_t* pend, int32_t g0, int32_t g1);
hipError_t launch_export_rows(const sim& s, int32_t net, int64_t i0, int64_t i1, int32_t* tgt,
                              uint8_t* dly, int16_t* wq, const int64_t* out_off);
hipError_t launch_quantise(const sim& s);
hipError_t launch_raster_bounds(const sim& s, int64_t t0, int64_t nsteps, int32_t lo, int32_t hi,
                                int64_t* bounds);
hipError_t launch_raster_take(const sim& s, int64_t nsteps, const int64_t* bounds,
                              const int64_t* dst_off, int32_t lo, int64_t n, int32_t* out);
hipError_t launch_raster_lengths(const sim& s, int64_t nsteps, const int64_t* bounds,
                                 int64_t* len);
hipError_t launch_adjoint_window(const sim& s, int64_t top, int64_t lo, const float* grad_rates,
                                 float scale, float beta, int64_t* next);
bool adjoint_col_fits(int32_t npc, int32_t d_min, int32_t d_max);
hipError_t prepare_adjoint_kernels();
hipError_t launch_reduce_parts(const sim& s, double* out);
hipError_t launch_canon_map(const sim& s, int mode, const float* src, float* dst);
hipError_t launch_canon_perm(const sim& s, uint16_t* rel);
hipError_t launch_weights_from_records(const sim& s);
hipError_t launch_column_rates(const sim& s, float scale, float* rates);
hipError_t launch_rate_loss(const sim& s, const float* rates, const float* targets, float* loss,
                            float* grad_rates);
hipError_t launch_fill_entries(const sim& s);
hipError_t launch_fill_dly(const sim& s);
hipError_t launch_rev_count(const sim& s, int32_t* cnt);
hipError_t launch_rev_fill(const sim& s, unsigned long long* fill);
hipError_t launch_stdp_post(const sim& s, const StepArgs& a, int64_t u);
hipError_t sort_rev(const sim& s, int64_t chunk, int32_t max_segs, uint64_t* alt, int32_t* off,
                    void* temp, size_t temp_bytes, const std::vector<int64_t>& h_ptr);
hipError_t sort_rev_temp_bytes(int64_t chunk, int32_t segs, size_t* bytes);
int64_t scan_scratch_len(int64_t n);

StepArgs make_step_args(const sim& s);
// the message sim_last_error(NULL) returns (calls that have no simulation handle)
void set_create_error(const std::string& msg);

}  // namespace dpsnn
