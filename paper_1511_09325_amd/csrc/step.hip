// step.hip -- the per-1 ms step on gfx950.
//
// The paper's simulator is mixed time- and event-driven (section 1): every neuron is
// integrated every step, and synaptic work is proportional to the spikes.  One step u:
//   input    A_j = (recurrent input due at step u) + n_j(u) * J_ext   (int32, 2^-16 mV)
//            n_j(u) ~ Poisson(ext_syn * rate * dt) from word j mod 4 of Philox at counter
//            (j / 4, u, 0, EXT), j the network-local index,
//            inverse CDF against 63 integer thresholds
//   neuron   refractory: count down, V = V_reset, input discarded;
//            else V~ = ((P_m V) - (gamma Ca)) + A 2^-16, spike if V~ >= theta, then
//            V = V_reset and the refractory counter is set; Ca = P_c Ca + alpha s
//            (LIF with calcium-driven AHP, section 2), float32, no contraction
//   spikes   ascending local ids per column (wave ballots + workgroup prefix)
//   delivery each synapse (delay d) of a spike at step u contributes at step u + d
//
// Two delivery strategies, bit-identical because the input is an integer sum:
//   ARRIVAL  a workgroup works on one tile of up to 4x4 target columns at a time (and takes
//            further tiles when there are more than the device holds workgroups).  At step
//            u it gathers, from the spike history of every column with synapses into the
//            tile, the delay group (i, d) of every neuron i that spiked at u - d, keeps the
//            synapses whose target lies in the tile, accumulates them in LDS with integer
//            atomics, then updates the tile's neurons -- one fused kernel, no ring in HBM.
//   PUSH     update kernel reading a delay ring ring[u % DH][j], then a delivery kernel
//            that scatters each spiking row into ring[(u + d) % DH][target] with
//            device-scope integer atomics.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "dpsnn_internal.h"

namespace dpsnn {
namespace {

constexpr int kMaxItems = kMaxTilePairs * kMaxDelay;
static_assert(kMaxItems + 1 >= 1024, "the tile order's buckets reuse the item prefix array");
constexpr int kPIF = 4;               // 16-byte synapse loads per lane in flight (plain mode)
constexpr int kIdxWords = (8 + 2 * (kMaxDelay + 2) + 15) / 16;  // 16-byte words of an entry

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Workgroup-wide exclusive scan: wave scans in registers, then the wave totals are scanned
// by the first wave (no per-wave branches, so no per-wave masks are kept live).
template <int BLOCK>
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t* total, int32_t* wsum) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int32_t v = lane < NW ? wsum[lane] : 0;
    int32_t c = v;
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const int32_t t = __shfl_up(c, off);
      if (lane >= off) c += t;
    }
    if (lane < NW) wsum[NW + lane] = c - v;  // exclusive prefix of the wave totals
    if (lane == NW - 1) wsum[2 * NW] = c;
  }
  __syncthreads();
  const int32_t before = wsum[NW + wave];
  *total = wsum[2 * NW];
  __syncthreads();
  return before + incl - x;
}

template <int BLOCK>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x,
                                                           unsigned long long* red) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
  if (lane == 0) red[wave] = x;
  __syncthreads();
  unsigned long long all = lane < NW ? red[lane] : 0ull;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) all += __shfl_down(all, off);
  all = __shfl(all, 0);
  __syncthreads();
  return all;
}

// Number of thresholds <= x (the thresholds are non-decreasing): a branch-free binary search
// of fixed depth, so that the searches of several neurons interleave.
static_assert(kPoissonEntries == 63, "six halvings cover the 63 thresholds");
__device__ __forceinline__ int32_t poisson_count(const uint64_t* tab, uint32_t x) {
  int pos = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (tab[pos + step - 1] <= (uint64_t)x) pos += step;
  return pos;
}

// One neuron's step from its state and input (no memory access).  MODEL (kModel*):
//   LIF:      refractory: count down, V = V_reset, input discarded; else
//             V~ = ((P_m V) - (gamma Ca)) + I [- (gamma_Na Na) before adding I with the
//             sodium variable], spike if V~ >= theta, then V = V_reset and the refractory
//             counter is set; Ca = P_c Ca + alpha s [Na = P_Na Na + alpha_Na s]
//   IZH:      two 0.5 ms Euler steps of v' = 0.04 v^2 + 5 v + 140 - u + I, then
//             u = u + a (b v - u); spike if v >= v_peak, then v = c, u = u + d (a, b, c, d of
//             the neuron's type; u is kept in the Ca array); no refractory period
// every operation float32, rounded, in this order (the build turns contraction off).
struct NeuronOut {
  float v, ca, na, vt;
  int32_t rf;
  bool spike, refr;
};

__device__ __forceinline__ float izh_half_step(float v, float u, float cur) {
  const float sq = v * v;
  const float quad = 0.04f * sq;
  const float lin = 5.0f * v;
  float rhs = quad + lin;
  rhs = rhs + 140.0f;
  rhs = rhs - u;
  rhs = rhs + cur;
  const float half = 0.5f * rhs;
  return v + half;
}

template <int MODEL>
__device__ __forceinline__ NeuronOut neuron_update(const StepArgs& a, int32_t rec_in, int32_t n_ext,
                                                  float vprev, float caprev, float naprev,
                                                  int32_t rf, bool excit) {
  const uint32_t asum = (uint32_t)rec_in + (uint32_t)n_ext * (uint32_t)a.k.jfx;
  const float cur = (float)(int32_t)asum * 0x1p-16f;
  NeuronOut o{0.0f, 0.0f, 0.0f, 0.0f, rf, false, false};
  if (MODEL == kModelIzh) {
    const float pa = excit ? a.k.ia[0] : a.k.ia[1], pb = excit ? a.k.ib[0] : a.k.ib[1];
    const float pc = excit ? a.k.ic[0] : a.k.ic[1], pd = excit ? a.k.id[0] : a.k.id[1];
    const float v1 = izh_half_step(vprev, caprev, cur);
    const float v2 = izh_half_step(v1, caprev, cur);
    const float bv = pb * v2;
    const float gap = bv - caprev;
    const float du = pa * gap;
    const float unew = caprev + du;
    o.vt = v2;
    o.rf = 0;
    if (v2 >= a.k.vpeak) {
      o.spike = true;
      o.v = pc;
      o.ca = unew + pd;
    } else {
      o.v = v2;
      o.ca = unew;
    }
    return o;
  }
  if (rf > 0) {
    o.refr = true;
    o.rf = rf - 1;
    o.v = a.k.vreset;
  } else {
    const float leak = a.k.pm * vprev;
    const float ahp = a.k.gam * caprev;
    float drop = leak - ahp;
    if (MODEL == kModelLifNa) {
      const float ahp_na = a.k.gna * naprev;
      drop = drop - ahp_na;
    }
    o.vt = drop + cur;
    if (o.vt >= a.k.theta) {
      o.spike = true;
      o.v = a.k.vreset;
      o.rf = a.k.tref;
    } else {
      o.v = o.vt;
    }
  }
  const float decayed = a.k.pc * caprev;
  o.ca = decayed + (o.spike ? a.k.alpha : 0.0f);
  if (MODEL == kModelLifNa) {
    const float na_decayed = a.k.pna * naprev;
    o.na = na_decayed + (o.spike ? a.k.alpha_na : 0.0f);
  }
  return o;
}

// Stores a neuron's new state (and its trajectory when recording: REC false compiles the
// recording out, for kernels that never run with it).
template <bool REC, int MODEL>
__device__ __forceinline__ void neuron_store(const StepArgs& a, int64_t j, int64_t u,
                                             const NeuronOut& o, float vprev, float caprev) {
  a.v[j] = o.v;
  a.ca[j] = o.ca;
  if (MODEL == kModelLifNa) a.na[j] = o.na;
  a.ref[j] = (uint8_t)o.rf;
  if (REC && a.rec_vprev) {
    const int64_t r = (u - a.rec_base) * (int64_t)a.n_cols * a.npc + j;
    a.rec_vprev[r] = vprev;
    a.rec_caprev[r] = caprev;
    a.rec_vt[r] = o.vt;
    a.rec_flags[r] = (uint8_t)((o.spike ? 1 : 0) | (o.refr ? 2 : 0));
  }
}

template <int MODEL>
__device__ __forceinline__ bool neuron_step(const StepArgs& a, int64_t j, int64_t u,
                                            int32_t rec_in, int32_t n_ext, float vprev,
                                            float caprev, int32_t rf, bool excit) {
  const float naprev = MODEL == kModelLifNa ? a.na[j] : 0.0f;
  const NeuronOut o = neuron_update<MODEL>(a, rec_in, n_ext, vprev, caprev, naprev, rf, excit);
  neuron_store<MODEL == kModelLif, MODEL>(a, j, u, o, vprev, caprev);
  return o.spike;
}

// The external count of neuron k of column g: one Philox block serves four consecutive
// network-local neurons jl, each taking word jl mod 4 of the block at counter (jl / 4, u).
__device__ __forceinline__ uint32_t block_word(const Rand4& x, uint32_t w) {
  return w == 0 ? x.x : w == 1 ? x.y : w == 2 ? x.z : x.w;
}

__device__ __forceinline__ int32_t external_count(const StepArgs& a, int32_t cloc, int k, int64_t u,
                                                  const uint64_t* ptab, uint32_t key0,
                                                  uint32_t key1) {
  const uint32_t jl = (uint32_t)(cloc * a.npc + k);
  const Rand4 x = philox10(jl >> 2, (uint32_t)u, 0u, kStreamExt, key0, key1);
  return poisson_count(ptab, block_word(x, jl & 3u));
}

// Delays read for spikes of age b (emitted at u - b): at a light step only the spikes
// emitted since the gathering step (b <= jnew), with delay b; at a gathering step with
// window W the delays b .. b + W - 1.  Clipped to [d_min, d_max].  Returns how many, and
// the first in *dlo.
__device__ __forceinline__ int32_t item_delays(const StepArgs& a, bool light, int32_t jnew,
                                               int32_t W, int32_t b, int32_t* dlo) {
  const int32_t d_max = a.d_min + a.nd - 1;
  int32_t lo = b, hi = b;
  if (light) {
    if (b > jnew) return 0;
  } else {
    hi = b + W - 1;
  }
  if (lo < a.d_min) lo = a.d_min;
  if (hi > d_max) hi = d_max;
  *dlo = lo;
  return hi >= lo ? hi - lo + 1 : 0;
}

// Order of the tile kernel's tiles: by decreasing synapse records read at the last gathering
// step, so that the largest tiles start first and the smallest fill the end (longest-first
// list scheduling); the spread of work between tiles follows the spatial spread of firing
// rates.  A counting sort over BLOCK buckets of the work scaled to the largest.  Workgroup b
// of a launch starts on XCD b mod 8, so the ranks are dealt to the XCDs in a snake (ranks
// 8k .. 8k + 7 to XCDs 0..7 for even k, 7..0 for odd k), which keeps their shares of the
// work even.  Run by one workgroup, after every other workgroup of the launch has finished;
// the results do not depend on the order.
template <int BLOCK>
__device__ void order_tiles(const StepArgs& a, int32_t* cnt, int32_t* wsum) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t mx = 0;
  for (int32_t t = tid; t < a.n_tiles; t += BLOCK)
    mx = max(mx, __hip_atomic_load(&a.tile_work[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int32_t)mx, off));
  if (lane == 0) wsum[wave] = (int32_t)mx;
  cnt[tid] = 0;
  __syncthreads();
  mx = 0;
  for (int w = 0; w < NW; ++w) mx = max(mx, (uint32_t)wsum[w]);
  const uint64_t den = (uint64_t)mx + 1;
  __syncthreads();
  for (int32_t t = tid; t < a.n_tiles; t += BLOCK) {
    const uint32_t w = __hip_atomic_load(&a.tile_work[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicAdd(&cnt[BLOCK - 1 - (int)((uint64_t)w * BLOCK / den)], 1);
  }
  __syncthreads();
  int32_t tot;
  const int32_t mine = cnt[tid];
  const int32_t ex = block_excl_scan<BLOCK>(mine, &tot, wsum);
  cnt[tid] = ex;
  __syncthreads();
  for (int32_t t = tid; t < a.n_tiles; t += BLOCK) {
    const uint32_t w = __hip_atomic_load(&a.tile_work[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t pos = atomicAdd(&cnt[BLOCK - 1 - (int)((uint64_t)w * BLOCK / den)], 1);
    if (((pos >> 3) & 1) && pos < (a.n_tiles & ~7)) pos ^= 7;  // odd full blocks of 8 reversed
    a.tile_order[pos] = t;
  }
  for (int32_t b = a.n_tiles + tid; b < a.grid_tiles; b += BLOCK) a.tile_order[b] = -1;
}

// ---- ARRIVAL: tiles of target columns ---------------------------------------------------
//
// Work list of a tile at step u: items (pair si, delay index dd) where a pair is a source
// column with synapses into the tile and the part of its rows that holds them (in the
// tiling the synapse store was built for, exactly the synapses into this tile); an item is
// the spike list of the source column at step u - d_min - dd, and every spike i of an item
// is one group: the contiguous synapses of (i, part, delay).  The groups are taken in
// batches of 64 per wave, without workgroup barriers: each lane locates one group (binary
// search over the item prefix, one spike id, one row-index entry), then each quad of lanes
// streams the four groups of its lanes in 16-byte words, keeping the synapses whose target
// column is in the tile (the record's rank, looked up in the pair's slot table) and adding
// them to the tile's LDS accumulators with integer atomics.  Then the tile's neurons are
// updated in 64-neuron chunks and the spikes compacted per column, in ascending order.
static_assert(kPoissonEntries <= 64, "one Poisson threshold per lane of the first wave");

template <int BLOCK, bool TRAIN, int MODEL, bool PLAST>
// At least four waves per SIMD for every workgroup size (at most 128 VGPRs), so that two
// 512-thread workgroups of the steps inside a window share a compute unit.
//
// PLAST (spike-timing-dependent plasticity; one step per gather, native tiling, so that every
// record read belongs to this tile and is read once): the postsynaptic traces of the tile's
// neurons, decayed to this step, sit in LDS beside the accumulators; every plastic record
// (weight >= 0) delivers its weight and is then depressed by rint(a_minus y- 2^14), floored
// at 0, and its 16-byte piece written back when a weight changed.  The update then writes
// the traces of this step (y = y- + s, x_u = P+ x_{u-1} + s).
__global__ __launch_bounds__(BLOCK, 4) void k_step_tile(StepArgs a, int64_t u_arg, int32_t maxc,
                                                     int32_t kacc) {
  const int64_t u = u_arg + (a.now_dev ? *a.now_dev : 0);
  constexpr int NW = BLOCK / 64;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ uint64_t ptab[kPoissonEntries];
  __shared__ int32_t it_pref[kMaxItems + 1];
  __shared__ int32_t s_src[kMaxTilePairs];      // source column of each pair
  __shared__ int32_t s_part[kMaxTilePairs];     // global part index of each pair
  __shared__ uint64_t s_slots[kMaxTilePairs];    // per pair: 5-bit tile slot of each rank
  __shared__ int32_t s_col[kMaxTileCols];
  __shared__ int32_t s_cloc[kMaxTileCols];      // index of each column within its network
  __shared__ uint32_t s_key[2];                 // the network's Philox key
  __shared__ int32_t s_cnp[kMaxTileCols];       // parts of each column
  __shared__ int32_t s_cpf[kMaxTileCols];       // first part index of each column
  __shared__ int32_t s_tot[kMaxTileCols];       // spikes of each column at this step
  __shared__ int32_t s_epre[kMaxTileCols + 1];  // prefix of (parts x spikes) over columns
  __shared__ int32_t s_next_bt;                 // next batch of the gather to be taken
  __shared__ int32_t wsum[2 * NW + 1];
  __shared__ unsigned long long red5[5][NW];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int npc = a.npc;
  const int nch = (npc + 63) >> 6;
  // dynamic LDS: acc[kacc][maxc*npc] | spike masks[maxc*nch] | counts[maxc*nch] (| PLAST:
  // decayed postsynaptic traces[maxc*npc]), kacc the accumulators this launch has room for
  // (the window's K, or 1 for a light step's launch)
  const int32_t K = a.gk;
  int32_t* acc = (int32_t*)lds;
  size_t off = ((size_t)kacc * maxc * npc * 4 + 15) & ~(size_t)15;
  unsigned long long* smask = (unsigned long long*)(lds + off);
  off += (size_t)maxc * nch * 8;
  int32_t* scnt = (int32_t*)(lds + off);
  off += ((size_t)maxc * nch * 4 + 15) & ~(size_t)15;
  float* ym = (float*)(lds + off);
  (void)ym;

  // Steps are gathered in windows of up to K: a gathering step reads, for every spike, the
  // delay groups due at its own step and at the following steps of its window (adjacent in
  // memory), keeping one accumulator per step; the accumulators of later steps go to
  // acc_save.  The other steps of the window ("light" steps) read only the spikes emitted
  // since the gathering step, plus their saved accumulator.  *gath is the last gathering
  // step (-1 after anything that invalidates acc_save).  A launch with room for fewer
  // accumulators than its window needs gathers its own step only and records no window.
  const int64_t g_last = *a.gath;
  const bool light = K > 1 && g_last >= 0 && u > g_last && u < g_last + (K - (int32_t)(g_last % K));
  const int32_t W = light ? 1 : min(K - (int32_t)(u % K), kacc);
  const bool full_window = K > 1 && !light && W == K - (int32_t)(u % K);
  const int32_t jnew = light ? (int32_t)(u - g_last) : 0;
  const int32_t NB = a.dh - 1;  // spike ages b = u - t in [1, d_max]
  const int64_t nall = (int64_t)a.n_cols * npc;
  const int32_t u_slot = (int32_t)(u % a.dh);
  const int64_t light_save = light ? (u % K) * nall : 0;  // this step's saved accumulator
  // Workgroup b runs entry b of tile_order.  With more tiles than the device holds
  // workgroups at once, the launch has only as many workgroups, and each one that finishes
  // takes the next entry from a device counter (gdone[1]): every compute unit takes the next
  // tile as soon as it is free, whichever XCD it sits in (list scheduling, largest measured
  // work first; the first round needs no counter, so that the launch does not start with
  // every workgroup contending for one address).  The last workgroup to finish resets it.
  const bool handout = (int32_t)gridDim.x < a.grid_tiles;
  __shared__ int32_t s_b;
  for (int32_t b_own = blockIdx.x;; b_own += gridDim.x) {
    int32_t b = b_own;
    if (handout && b_own >= (int32_t)gridDim.x) {
      if (tid == 0) s_b = (int32_t)gridDim.x + (int32_t)atomicAdd(a.gdone + 1, 1u);
      __syncthreads();
      b = s_b;
      __syncthreads();
    }
    if (b >= a.grid_tiles) break;
    const int32_t tile = a.tile_order[b];
    if (tile < 0) continue;
    const int T = a.tile_ncols[tile];
    // the tile's pieces, addressed relative to the first piece of its source rows (train
    // mode, whose stores stay below 2^32 pieces, addresses them from the store's start)
    const int64_t tbase = TRAIN ? 0 : a.tile_base[tile];
    const uint32_t* syn_t = a.syn + 4 * tbase;
    uint32_t* syn_rw_t = PLAST ? a.syn_rw + 4 * tbase : nullptr;
    (void)syn_rw_t;
    const int ns = a.tile_npairs[tile];
    if (tid < kMaxTileCols) {
      const int4 ci = a.tile_cinfo[tile * kMaxTileCols + tid];
      s_col[tid] = ci.x;
      s_cloc[tid] = ci.y;
      s_cnp[tid] = ci.z;
      s_cpf[tid] = ci.w;
    }
    if (tid < kMaxTilePairs) {
      const int2 pi = a.tile_pinfo[tile * kMaxTilePairs + tid];
      s_src[tid] = pi.x;
      s_part[tid] = pi.y;
      s_slots[tid] = a.tile_slots[tile * kMaxTilePairs + tid];
    }
    // the network's Poisson table and key, needed from the update on: loaded now, stored
    // to LDS after the item prefix so that the load overlaps it
    const int32_t net = a.tile_net[tile];
    const uint64_t ptab_q = tid < kPoissonEntries ? a.net_ptab[(int64_t)net * kPoissonEntries + tid] : 0;
    const uint32_t key_q = tid < 2 ? a.net_key[2 * net + tid] : 0u;
    const int32_t TN = T * npc;
    for (int e = tid; e < W * TN; e += BLOCK) acc[e] = 0;
    __syncthreads();
    if (PLAST) {
      for (int e = tid; e < TN; e += BLOCK) {
        const int col = e / npc;
        ym[e] = a.sp_pm * a.sp_y[(int64_t)s_col[col] * npc + (e - col * npc)];
      }
    }
    // 1. items (pair, spike age b) and their group counts: spikes x delays read
    const int n_items = ns * NB;
    int32_t carry = 0;
    for (int bb = 0; bb < n_items; bb += BLOCK) {
      const int it = bb + tid;
      int32_t cnt = 0;
      if (it < n_items) {
        const int si = it / NB, ag = it - si * NB + 1;
        const int64_t t = u - ag;
        int32_t dlo;
        const int32_t ndel = item_delays(a, light, jnew, W, ag, &dlo);
        int32_t slot = u_slot - ag;
        if (slot < 0) slot += a.dh;
        if (t >= 0 && ndel > 0) cnt = ndel * a.hist_cnt[(int64_t)slot * a.n_cols + s_src[si]];
      }
      int32_t tot;
      const int32_t ex = block_excl_scan<BLOCK>(cnt, &tot, wsum);
      if (it < n_items) it_pref[it] = carry + ex;
      carry += tot;
    }
    if (tid == 0) it_pref[n_items] = carry;
    if (tid == 0) s_next_bt = NW;
    if (tid < kPoissonEntries) ptab[tid] = ptab_q;
    if (tid < 2) s_key[tid] = key_q;
    __syncthreads();
    const int32_t total = carry;
    unsigned long long streamed = 0;
    uint32_t delivered = 0;
    // 2. gather.  Each wave independently takes batches of 64 groups (group q of the tile's
    // list is spike q - it_pref[item] of item `item`): every lane locates one group, then
    // every quad of lanes streams the four groups of its lanes in 16-byte pieces, kPIF
    // loads in flight per lane, and adds the synapses into the LDS accumulators.
    const int quad0 = lane & ~3, ql = lane & 3;
    const uint32_t npc4 = (uint32_t)npc * 4u;
    uint32_t dlane = 0;  // records delivered by this lane (a register add per record)
    // exact small-integer quotients through float reciprocals (operands < 2^16)
    const float inv_nb = 1.0f / (float)NB;
    // A lane's group of a batch: its pair, the step offset of its accumulator, its spike's
    // part start and the group's first and end offsets within the part (the three loads).
    // The next batch is located (and its loads issued) before the current one is streamed,
    // so that the two latencies overlap.
    struct Located {
      int32_t si, gsb, g0, g1;
      uint32_t st;
    };
    auto locate = [&](int32_t bt) {
      Located L{0, 0, 0, 0, 0u};
      const int32_t qq = bt * 64 + lane;
      if (qq < total) {
        int lo = 0, hi = n_items;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (it_pref[mid] <= qq) lo = mid;
          else hi = mid;
        }
        const int si = (int)(((float)lo + 0.5f) * inv_nb);
        const int ag = lo - si * NB + 1;
        int32_t dlo;
        const int32_t ndel = item_delays(a, light, jnew, W, ag, &dlo);
        const int32_t r = qq - it_pref[lo];
        const int32_t pos = (int32_t)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)ndel));
        const int32_t d = dlo + (r - pos * ndel);
        int32_t slot = u_slot - ag;
        if (slot < 0) slot += a.dh;
        const int64_t pid = (int64_t)slot * a.n_parts + s_part[si];
        const uint16_t* go = a.hist_go + (pid * (a.nd + 1) + (d - a.d_min)) * npc + pos;
        L.si = si;
        L.gsb = (d - ag) * TN * 4;
        L.g0 = go[0];
        L.g1 = go[npc];
        L.st = (uint32_t)(a.hist_st[pid * npc + pos] - (uint64_t)tbase);
      }
      return L;
    };
    int32_t bt = wave;
    Located cur = locate(bt);
    while (bt * 64 < total) {
      // the wave's next batch (the atomic's latency hides under the search), located now
      int32_t bt_next = 0;
      if (lane == 0) bt_next = atomicAdd(&s_next_bt, 1);
      bt_next = __shfl(bt_next, 0);
      const Located nxt = locate(bt_next);
      // this lane's group: first 16-byte piece, length in pieces, the offset of the
      // accumulator of its step and its pair's slot word
      const bool has = bt * 64 + lane < total;
      const uint32_t gpc = cur.st + ((uint32_t)cur.g0 >> 2);
      const int32_t glen = has ? (cur.g1 - cur.g0) >> 2 : 0;
      const int32_t gsb = cur.gsb;
      const uint64_t gsl = has ? s_slots[cur.si] : ~(uint64_t)0;
      streamed += (unsigned long long)(glen * 4);
      // the quad streams the pieces of its four groups: piece p of the quad lies in group m
      // where pref[m] <= p < pref[m + 1], at piece index bias[m] + p; sbq is the byte offset
      // of the group's step accumulator
      int32_t pref[5], sbq[4];
      uint32_t bias[4];
      uint64_t slq[4];
      pref[0] = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        bias[m] = (uint32_t)__shfl((int32_t)gpc, quad0 + m) - (uint32_t)pref[m];
        sbq[m] = __shfl(gsb, quad0 + m);
        slq[m] = ((uint64_t)(uint32_t)__shfl((int32_t)(gsl >> 32), quad0 + m) << 32) |
                 (uint32_t)__shfl((int32_t)(uint32_t)gsl, quad0 + m);
        pref[m + 1] = pref[m] + __shfl(glen, quad0 + m);
      }
      const int32_t npieces = pref[4];
      // train mode carries each piece's four efficacies as well: two pieces in flight keep
      // its registers from spilling (measured faster than one, three or four)
      constexpr int PIF = TRAIN ? 2 : kPIF;
      for (int32_t p0 = ql; p0 < npieces; p0 += 4 * PIF) {
        uint4 w[PIF];
        int32_t v[PIF][4];
        int32_t aoff[PIF];
        uint64_t sw[PIF];
        uint64_t pc[PIF];
#pragma unroll
        for (int q = 0; q < PIF; ++q) {
          const int32_t p = p0 + 4 * q;
          const bool valid = p < npieces;
          const bool m1 = p >= pref[1], m2 = p >= pref[2], m3 = p >= pref[3];
          const uint32_t b = m3 ? bias[3] : m2 ? bias[2] : m1 ? bias[1] : bias[0];
          aoff[q] = m3 ? sbq[3] : m2 ? sbq[2] : m1 ? sbq[1] : sbq[0];
          sw[q] = m3 ? slq[3] : m2 ? slq[2] : m1 ? slq[1] : slq[0];
          w[q] = make_uint4(kDummyRecord, kDummyRecord, kDummyRecord, kDummyRecord);
          pc[q] = 0;
          if (valid) {
            const uint64_t piece = (uint64_t)(b + (uint32_t)p);
            pc[q] = piece;
            w[q] = *(const uint4*)(syn_t + 4 * piece);
            if (TRAIN) *(int4*)&v[q][0] = *(const int4*)(a.wfx + 4 * piece);
          }
        }
        // tile slot of each record from its pair's slot word (rank r in bits 5r..5r+4; the
        // bits from the tenth field up are set, so dummies and absent ranks read 31); the
        // weights are added in their 2^-14 mV units (train mode: the float efficacies, in
        // 2^-16 mV), each lane counting the records it delivers
#pragma unroll
        for (int q = 0; q < PIF; ++q) {
          const uint32_t x[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t sl = (uint32_t)(sw[q] >> (5u * rec_rank(x[e]))) & 31u;
            const bool in = sl != (uint32_t)kNoSlot;
            dlane += in ? 1u : 0u;
            if (in) {
              const uint32_t off = __umul24(sl, npc4) + (uint32_t)aoff[q] + (rec_k(x[e]) << 2);
              atomicAdd((int32_t*)((unsigned char*)acc + off), TRAIN ? v[q][e] : rec_wq(x[e]));
            }
          }
          if (PLAST) {
            // depression of the plastic records just delivered (the piece's records all
            // belong to this tile; dummies read slot 31)
            uint32_t nw[4] = {x[0], x[1], x[2], x[3]};
            bool changed = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const uint32_t sl = (uint32_t)(sw[q] >> (5u * rec_rank(x[e]))) & 31u;
              const int32_t q0 = rec_wq(x[e]);
              if (sl != (uint32_t)kNoSlot && q0 >= 0) {
                const float yv = *(const float*)((const unsigned char*)ym + __umul24(sl, npc4) +
                                                 (rec_k(x[e]) << 2));
                const float t1 = a.sp_am * yv;
                const int32_t dq = (int32_t)__builtin_rintf(t1 * 16384.0f);
                if (dq != 0) {
                  nw[e] = (x[e] & 0xffffu) | ((uint32_t)max(q0 - dq, 0) << 16);
                  changed = true;
                }
              }
            }
            if (changed) *(uint4*)(syn_rw_t + 4 * pc[q]) = make_uint4(nw[0], nw[1], nw[2], nw[3]);
          }
        }
      }
      bt = bt_next;
      cur = nxt;
    }
    delivered = dlane;
    __syncthreads();
    // the accumulators of the later steps of the window, for their light steps
    for (int w = 1; w < W; ++w) {
      int32_t* dst = a.acc_save + ((u + w) % K) * nall;
      for (int c = wave; c < T * nch; c += NW) {
        const int col = c / nch, k = (c - col * nch) * 64 + lane;
        if (k < npc) dst[(int64_t)s_col[col] * npc + k] = acc[w * TN + col * npc + k];
      }
    }
    // 3. update, in rounds of four 64-neuron chunks of one column: chunk c is column c / nch,
    // neurons (c % nch) * 64 + lane.  When the column size is a multiple of 4, the 256
    // neurons of a round draw their external counts from 64 Philox blocks, one per lane,
    // handed to the neurons by lane shuffles; otherwise each lane draws its own block.
    const int nchunks = T * nch;
    const int nr = (nch + 3) >> 2;
    const bool shared_draw = (npc & 3) == 0;
    const uint32_t key0 = s_key[0], key1 = s_key[1];
    unsigned long long my_ext = 0, my_rec = 0;
    for (int rd = wave; rd < T * nr; rd += NW) {
      const int col = rd / nr, q0 = (rd - col * nr) * 4;
      const int32_t g = s_col[col];
      float vv[4], cc[4], na4[4], xp[4];
      int32_t rr[4], nx[4], sv[4];
      bool ok[4];
      const int32_t x_prev_slot = u_slot == 0 ? a.dh - 1 : u_slot - 1;
      // every global load of the round first, so that their latencies overlap: state and, at
      // a light step, the saved input
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = (q0 + m) * 64 + lane;
        ok[m] = q0 + m < nch && k < npc;
        vv[m] = 0.0f;
        cc[m] = 0.0f;
        na4[m] = 0.0f;
        xp[m] = 0.0f;
        rr[m] = 0;
        sv[m] = 0;
        if (ok[m]) {
          const int64_t j = (int64_t)g * npc + k;
          vv[m] = a.v[j];
          cc[m] = a.ca[j];
          if (MODEL == kModelLifNa) na4[m] = a.na[j];
          rr[m] = a.ref[j];
          if (light) sv[m] = a.acc_save[light_save + j];
          if (PLAST) xp[m] = a.sp_x[(int64_t)x_prev_slot * nall + j];
        }
      }
      const int32_t cloc = s_cloc[col];
      Rand4 blk{0u, 0u, 0u, 0u};
      if (shared_draw)
        blk = philox10(((uint32_t)(cloc * npc + q0 * 64) >> 2) + (uint32_t)lane,
                       (uint32_t)u, 0u, kStreamExt, key0, key1);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        nx[m] = 0;
        if (shared_draw) {
          const int src = 16 * m + (lane >> 2);
          const Rand4 b{(uint32_t)__shfl((int32_t)blk.x, src), (uint32_t)__shfl((int32_t)blk.y, src),
                        (uint32_t)__shfl((int32_t)blk.z, src), (uint32_t)__shfl((int32_t)blk.w, src)};
          if (ok[m]) nx[m] = poisson_count(ptab, block_word(b, (uint32_t)lane & 3u));
        } else if (ok[m]) {
          nx[m] = external_count(a, cloc, (q0 + m) * 64 + lane, u, ptab, key0, key1);
        }
      }
      // the four chunks' new states, then their stores (no load waits behind a store)
      NeuronOut o[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = (q0 + m) * 64 + lane;
        // accumulated recurrent input, to 2^-16 mV (train mode accumulates in those units)
        const uint32_t ai = (uint32_t)acc[col * npc + k] + (uint32_t)sv[m];
        const int32_t in = ok[m] ? (int32_t)(TRAIN ? ai : ai << 2) : 0;
        o[m] = neuron_update<MODEL>(a, in, nx[m], vv[m], cc[m], na4[m], rr[m], k < a.n_exc);
        o[m].spike = o[m].spike && ok[m];
        if (ok[m]) my_ext += (unsigned long long)nx[m];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (q0 + m < nch) {
          const int c = col * nch + q0 + m;
          if (ok[m])
            neuron_store<TRAIN, MODEL>(a, (int64_t)g * npc + (q0 + m) * 64 + lane, u, o[m], vv[m], cc[m]);
          if (PLAST && ok[m]) {
            const int k = (q0 + m) * 64 + lane;
            const int64_t j = (int64_t)g * npc + k;
            const float sp = o[m].spike ? 1.0f : 0.0f;
            a.sp_y[j] = ym[col * npc + k] + sp;
            const float decayed = a.sp_pp * xp[m];
            a.sp_x[(int64_t)u_slot * nall + j] = decayed + sp;
          }
          const unsigned long long bal = __ballot(o[m].spike);
          if (lane == 0) {
            smask[c] = bal;
            scnt[c] = __popcll(bal);
          }
        }
      }
    }
    __syncthreads();
    // 4. compaction: ascending ids of each column into the history slot of step u.  One
    // wave per column turns the per-chunk spike counts into exclusive offsets (nch <= 64).
    const int32_t slot_u = u_slot;
    const unsigned long long lt = lanemask_lt(lane);
    for (int col = wave; col < T; col += NW) {
      const int32_t x = lane < nch ? scnt[col * nch + lane] : 0;
      int32_t incl = x;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      if (lane < nch) scnt[col * nch + lane] = incl - x;
      if (lane == 63) s_tot[col] = incl;
    }
    __syncthreads();
    // the ids also go to LDS (over the accumulators, no longer needed) for the entries below
    uint16_t* s_ids = (uint16_t*)acc;
    for (int c = wave; c < nchunks; c += NW) {
      const int col = c / nch, first = col * nch;
      const unsigned long long m = smask[c];
      if ((m >> lane) & 1ull) {
        const int32_t pos = scnt[c] + __popcll(m & lt);
        const uint16_t id = (uint16_t)((c - first) * 64 + lane);
        a.hist_ids[((int64_t)slot_u * a.n_cols + s_col[col]) * npc + pos] = id;
        s_ids[col * npc + pos] = id;
      }
    }
    unsigned long long my_spk = 0;
    if (tid < T) {
      const int32_t tot = s_tot[tid];
      a.hist_cnt[(int64_t)slot_u * a.n_cols + s_col[tid]] = tot;
      if (tot) atomicAdd(&a.col_spk[s_col[tid]], (unsigned long long)tot);
      my_spk = (unsigned long long)tot;
    }
    __syncthreads();
    // 5. history entries of the step's spikes: one lane per (column, part, spike) copies the
    // part's row-index entry (loaded once) into the rows of the history, consecutive lanes
    // writing consecutive spike positions of each row
    if (tid == 0) {
      int32_t run = 0;
      for (int col = 0; col < T; ++col) {
        s_epre[col] = run;
        run += s_cnp[col] * s_tot[col];
      }
      s_epre[T] = run;
    }
    __syncthreads();
    for (int32_t e = tid; e < s_epre[T]; e += BLOCK) {
      int col = 0;
      while (col + 1 < T && s_epre[col + 1] <= e) ++col;
      const int32_t cnt = s_tot[col];
      const int32_t r = e - s_epre[col];
      const int p = r / cnt, pos = r - p * cnt;
      const int32_t k = s_ids[col * npc + pos];
      // entry (column's first entry npc * first part) + k * parts + p; every word is loaded
      // (the ones past the entry repeat its last word), so that the loads leave together
      const uint4* ent = (const uint4*)(a.idx + ((int64_t)npc * s_cpf[col] + (int64_t)k * s_cnp[col] + p) * a.idxw);
      const int nw = a.idxw >> 4;
      uint4 buf[kIdxWords];
#pragma unroll
      for (int q = 0; q < kIdxWords; ++q) buf[q] = ent[q < nw ? q : nw - 1];
      const int64_t pid = (int64_t)slot_u * a.n_parts + s_cpf[col] + p;
      a.hist_st[pid * npc + pos] = (uint64_t)(*(const int64_t*)&buf[0] >> 2);
      const uint16_t* go = (const uint16_t*)&buf[0] + 4;
      uint16_t* out = a.hist_go + pid * (int64_t)(a.nd + 1) * npc + pos;
#pragma unroll
      for (int f = 0; f <= kMaxDelay + 1; ++f) {
        if (f <= a.nd) out[(int64_t)f * npc] = go[f];
        if (f == a.nd + 1) my_rec += (unsigned long long)go[f];  // the part's synapses
      }
    }
    // the tile's counters: wave sums, then one sum per counter
    unsigned long long cv[5] = {my_spk, my_rec, my_ext, streamed, (unsigned long long)delivered};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) cv[q] += __shfl_down(cv[q], off);
      if (lane == 0) red5[q][wave] = cv[q];
    }
    __syncthreads();
    if (tid < 5) {
      unsigned long long all = 0;
      for (int w = 0; w < NW; ++w) all += red5[tid][w];
      if (all) atomicAdd(&a.net_cnt[kCounters * net + tid], all);
      if (tid == 0 && !light) {
        unsigned long long rd = 0;
        for (int w = 0; w < NW; ++w) rd += red5[3][w];
        a.tile_work[tile] = (uint32_t)min(rd, 0xffffffffull);
      }
    }
    __syncthreads();
  }
  // The last workgroup to finish resets the tile counter; after a gathering step it also
  // records the step (every workgroup has read *gath) and orders the tiles by the work just
  // measured for the following steps, which the other workgroups' release fences publish.
  // A light step without the counter needs none of this.
  if (!light || handout) {
    __shared__ int32_t s_last;
    if (tid == 0) {
      if (!light) __threadfence();
      s_last = atomicAdd(a.gdone, 1u) == gridDim.x - 1;
      if (s_last) {
        if (!light && full_window) *a.gath = u;
        a.gdone[1] = 0u;
        a.gdone[0] = 0u;
        __threadfence();
      }
    }
    __syncthreads();
    if (!light && s_last && a.order_by_work) order_tiles<BLOCK>(a, it_pref, wsum);
  }
}

// ---- PUSH: update from the ring, then scatter ------------------------------------------------
template <int BLOCK, int MODEL>
__global__ __launch_bounds__(BLOCK) void k_update_push(StepArgs a, int64_t u_arg) {
  const int64_t u = u_arg + (a.now_dev ? *a.now_dev : 0);
  constexpr int NW = BLOCK / 64;
  __shared__ uint64_t ptab[kPoissonEntries];
  __shared__ int32_t wcnt[NW];
  __shared__ unsigned long long red[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = lanemask_lt(lane);
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  int32_t* in = a.ring + (u % a.dh) * nall;
  const int32_t slot_u = (int32_t)(u % a.dh);
  for (int32_t b = blockIdx.x; b < a.grid_cols; b += gridDim.x) {
    const int32_t g = a.col_order[b];
    if (g < 0) continue;
    const int32_t net = a.col_net[g];
    for (int q = threadIdx.x; q < kPoissonEntries; q += BLOCK)
      ptab[q] = a.net_ptab[(int64_t)net * kPoissonEntries + q];
    __syncthreads();
    const uint32_t key0 = a.net_key[2 * net], key1 = a.net_key[2 * net + 1];
    uint16_t* out = a.hist_ids + ((int64_t)slot_u * a.n_cols + g) * a.npc;
    int32_t running = 0;
    unsigned long long my_ext = 0, my_rec = 0;
    for (int k0 = 0; k0 < a.npc; k0 += BLOCK) {
      const int k = k0 + (int)threadIdx.x;
      bool sp = false;
      if (k < a.npc) {
        const int64_t j = (int64_t)g * a.npc + k;
        const int32_t x = in[j];
        in[j] = 0;
        const int32_t nx = external_count(a, a.col_local[g], k, u, ptab, key0, key1);
        sp = neuron_step<MODEL>(a, j, u, x, nx, a.v[j], a.ca[j], a.ref[j], k < a.n_exc);
        my_ext += (unsigned long long)nx;
        if (sp) my_rec += (unsigned long long)a.deg[j];
      }
      const unsigned long long m = __ballot(sp);
      if (lane == 0) wcnt[wave] = __popcll(m);
      __syncthreads();
      int32_t before = 0, tot = 0;
      for (int w = 0; w < NW; ++w) {
        if (w < wave) before += wcnt[w];
        tot += wcnt[w];
      }
      if (sp) {
        const int32_t pos = running + before + __popcll(m & lt);
        out[pos] = (uint16_t)k;
        write_entries(a, g, k, slot_u, pos);
      }
      running += tot;
      __syncthreads();
    }
    const unsigned long long ext_all = block_sum_u64<BLOCK>(my_ext, red);
    const unsigned long long rec_all = block_sum_u64<BLOCK>(my_rec, red);
    if (threadIdx.x == 0) {
      a.hist_cnt[(int64_t)slot_u * a.n_cols + g] = running;
      if (running) a.col_spk[g] += (unsigned long long)running;
      atomicAdd(&a.net_cnt[kCounters * net + 0], (unsigned long long)running);
      atomicAdd(&a.net_cnt[kCounters * net + 1], rec_all);
      atomicAdd(&a.net_cnt[kCounters * net + 2], ext_all);
    }
    __syncthreads();
  }
}

template <int BLOCK, bool TRAIN>
__global__ __launch_bounds__(BLOCK) void k_deliver_push(StepArgs a, int64_t u_arg) {
  const int64_t u = u_arg + (a.now_dev ? *a.now_dev : 0);
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int32_t uslot = (int32_t)(u % a.dh);
  for (int32_t g = blockIdx.x; g < a.n_cols; g += gridDim.x) {
    const int32_t ns = a.hist_cnt[(int64_t)uslot * a.n_cols + g];
    const uint16_t* ids = a.hist_ids + ((int64_t)uslot * a.n_cols + g) * a.npc;
    const int np = a.col_np[g];
    for (int32_t q = wave; q < ns; q += NW) {
      const int32_t k = ids[q];
      const int64_t i = (int64_t)g * a.npc + k;
      const int32_t len = a.deg[i];
      if (lane == 0 && len) atomicAdd(&a.net_cnt[kCounters * a.col_net[g] + 3], (unsigned long long)len);
      for (int p = 0; p < np; ++p) {
        const uint8_t* ent = idx_entry(a, g, k, p);
        const int64_t st = ent_start(ent);
        const uint16_t* go = ent_goff(ent);
        const int32_t* pcol = a.part_col + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
        for (int dd = 0; dd < a.nd; ++dd) {
          int64_t slot = uslot + a.d_min + dd;
          if (slot >= a.dh) slot -= a.dh;
          for (int32_t f = go[dd] + lane; f < go[dd + 1]; f += 64) {
            const uint32_t w = a.syn[st + f];
            if (rec_rank(w) == (uint32_t)kDummyRank) continue;
            const int32_t tc = pcol[rec_rank(w)];
            atomicAdd(&a.ring[slot * nall + (int64_t)tc * a.npc + rec_k(w)],
                      TRAIN ? a.wfx[st + f] : rec_w32(w));
          }
        }
      }
    }
  }
}

// ---- state initialisation from Philox at (j, 0, 0, INIT) ------------------------------------
// LIF: V uniform on [0, V_reset), Ca = 0 (Na = 0).  Izhikevich: v uniform on [c, c + 5) mV,
// u = b v (the resting relation), with c, b of the neuron's type.
__global__ void k_init_state(StepArgs a, int32_t model) {
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nall;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = (int32_t)(j / a.npc);
    const int32_t k = (int32_t)(j - (int64_t)g * a.npc);
    const int32_t net = a.col_net[g];
    const Rand4 r = philox10((uint32_t)(a.col_local[g] * a.npc + k), 0u, 0u, kStreamInit,
                             a.net_key[2 * net], a.net_key[2 * net + 1]);
    const float unit = (float)(r.x >> 8) * 0x1p-24f;
    if (model == kModelIzh) {
      const bool excit = k < a.n_exc;
      const float spread = 5.0f * unit;
      const float v = (excit ? a.k.ic[0] : a.k.ic[1]) + spread;
      a.v[j] = v;
      a.ca[j] = (excit ? a.k.ib[0] : a.k.ib[1]) * v;
    } else {
      a.v[j] = a.k.vreset * unit;
      a.ca[j] = 0.0f;
    }
    if (a.na) a.na[j] = 0.0f;
    a.ref[j] = 0;
  }
}

// Workgroups of one kernel that device `dev` holds at once: its compute units times the
// workgroups of `block` threads with `lds` bytes of dynamic LDS that fit on one (cached per
// device, kernel and LDS size; 0 when the query fails, which is not cached, so that a later
// call asks again).
static int resident_workgroups(int dev, const void* fn, int block, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, fn, lds);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, n_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      per_cu <= 0 || n_cu <= 0) {
    (void)hipGetLastError();  // a failed query leaves no error for the launch to report
    return 0;
  }
  return cache[key] = per_cu * n_cu;
}

template <int BLOCK, bool TRAIN, int MODEL, bool PLAST>
void launch_tile_k(const sim& s, const StepArgs& a, int64_t u, int32_t kacc, size_t lds) {
  const void* fn = (const void*)k_step_tile<BLOCK, TRAIN, MODEL, PLAST>;
  const int res = resident_workgroups(s.device, fn, BLOCK, lds);
  const int32_t nwg = res > 0 ? std::min(s.grid_tiles, res) : s.grid_tiles;
  hipLaunchKernelGGL((k_step_tile<BLOCK, TRAIN, MODEL, PLAST>), dim3(std::max(nwg, 1)), dim3(BLOCK),
                     lds, s.stream, a, u, s.tile_max_cols, kacc);
}

template <int BLOCK, bool PLAST>
void launch_tile_p(const sim& s, const StepArgs& a, int64_t u, int32_t kacc, bool train) {
  const size_t lds = tile_lds_bytes(s, kacc);
  if (train)  // train mode runs the LIF neuron with one AHP variable only
    launch_tile_k<BLOCK, true, kModelLif, false>(s, a, u, kacc, lds);
  else if (s.model == kModelLifNa)
    launch_tile_k<BLOCK, false, kModelLifNa, PLAST>(s, a, u, kacc, lds);
  else if (s.model == kModelIzh)
    launch_tile_k<BLOCK, false, kModelIzh, PLAST>(s, a, u, kacc, lds);
  else
    launch_tile_k<BLOCK, false, kModelLif, PLAST>(s, a, u, kacc, lds);
}

template <int BLOCK>
void launch_tile(const sim& s, const StepArgs& a, int64_t u, int32_t kacc, bool train) {
  if (s.cfg.stdp) {
    launch_tile_p<BLOCK, true>(s, a, u, kacc, false);
    (void)launch_stdp_post(s, a, u);
  } else {
    launch_tile_p<BLOCK, false>(s, a, u, kacc, train);
  }
}

template <int BLOCK>
hipError_t launch_step_b(sim& s, int64_t u, int32_t delivery, int part) {
  const StepArgs a = make_step_args(s);
  const bool train = s.wfx != nullptr;
  if (delivery == DPSNN_DELIVERY_ARRIVAL) {
    if (part == 1) return hipSuccess;
    if (s.rec_on && !train) return hipErrorInvalidValue;  // only the train kernel records
    // Steps inside a gather window (u mod K != 0) are light: their launch reserves one
    // accumulator and uses workgroups of at most 512 threads, so that two tiles share a
    // compute unit and hide each other's latencies.  (Should the window not be valid on
    // the device, such a launch gathers its own step alone.)
    const int64_t uabs = s.graph_mode ? s.graph_base + u : u;
    if (s.gk > 1 && uabs % s.gk != 0) {
      if (BLOCK > 512) launch_tile<512>(s, a, u, 1, train);
      else launch_tile<BLOCK>(s, a, u, 1, train);
    } else {
      launch_tile<BLOCK>(s, a, u, s.gk, train);
    }
    return hipGetLastError();
  }
  if (part != 1) {
    if (s.model == kModelLifNa)
      hipLaunchKernelGGL((k_update_push<BLOCK, kModelLifNa>), dim3(s.grid_cols), dim3(BLOCK), 0,
                         s.stream, a, u);
    else if (s.model == kModelIzh)
      hipLaunchKernelGGL((k_update_push<BLOCK, kModelIzh>), dim3(s.grid_cols), dim3(BLOCK), 0,
                         s.stream, a, u);
    else
      hipLaunchKernelGGL((k_update_push<BLOCK, kModelLif>), dim3(s.grid_cols), dim3(BLOCK), 0,
                         s.stream, a, u);
  }
  if (part != 0) {
    if (train)
      hipLaunchKernelGGL((k_deliver_push<BLOCK, true>), dim3(s.n_cols), dim3(BLOCK), 0, s.stream, a, u);
    else
      hipLaunchKernelGGL((k_deliver_push<BLOCK, false>), dim3(s.n_cols), dim3(BLOCK), 0, s.stream, a, u);
  }
  return hipGetLastError();
}

}  // namespace

// LDS of the tile kernel: accumulators and spike masks of the largest tile (dynamic), plus
// the kernel's static tables; together at most the 160 KB of a workgroup.
static size_t tile_fixed_lds(const sim& s, int32_t kacc) {
  const size_t nch = (size_t)(s.npc + 63) / 64;
  size_t b = ((size_t)std::max(kacc, 1) * s.tile_max_cols * s.npc * 4 + 15) & ~(size_t)15;
  b += (size_t)s.tile_max_cols * nch * 8;
  b += ((size_t)s.tile_max_cols * nch * 4 + 15) & ~(size_t)15;
  if (s.cfg.stdp) b += (size_t)s.tile_max_cols * s.npc * 4;  // decayed postsynaptic traces
  return b;
}

static size_t tile_static_bytes() {
  return sizeof(uint64_t) * kPoissonEntries + sizeof(int32_t) * (kMaxItems + 1) +
         (sizeof(int32_t) * 2 + sizeof(uint64_t)) * kMaxTilePairs + sizeof(int32_t) * 3 * kMaxTileCols +
         (sizeof(int32_t) * 2 + 1 + 5 * sizeof(uint64_t)) * 16 + 64;
}

// The static LDS of the tile kernels as the compiler laid it out (the largest of their
// instantiations), read at set-up; the estimate above until then.
static size_t g_tile_static_lds = 0;

bool tile_lds_ok(const sim& s) {
  const size_t fixed = g_tile_static_lds ? g_tile_static_lds : tile_static_bytes() + 1024;
  return tile_fixed_lds(s, s.gk) + fixed <= kMaxLds;
}

size_t tile_lds_bytes(const sim& s, int32_t kacc) { return tile_fixed_lds(s, kacc); }

StepArgs make_step_args(const sim& s) {
  StepArgs a{};
  a.npc = s.npc;
  a.nd = s.nd;
  a.d_min = s.cfg.d_min;
  a.dh = s.dh;
  a.n_cols = s.n_cols;
  a.idxw = s.idxw;
  a.n_exc = s.cfg.n_exc;
  a.now_dev = s.graph_mode ? s.d_now : nullptr;
  a.col_net = s.col_net;
  a.col_local = s.col_local;
  a.col_nbr = s.col_nbr;
  a.col_nn = s.col_nn;
  a.col_order = s.col_order;
  a.grid_cols = s.grid_cols;
  a.net_key = s.net_key;
  a.net_ptab = s.net_ptab;
  a.tile_order = s.tile_order;
  a.grid_tiles = s.grid_tiles;
  a.n_tiles = s.n_tiles;
  a.tile_work = s.tile_work;
  a.order_by_work = s.order_by_work;
  a.tile_cinfo = (const int4*)s.tile_cinfo;
  a.tile_ncols = s.tile_ncols;
  a.tile_pinfo = (const int2*)s.tile_pinfo;
  a.tile_net = s.tile_net;
  a.tile_base = s.tile_base;
  a.tile_npairs = s.tile_npairs;
  a.col_np = s.col_np;
  a.col_part = s.col_part;
  a.col_pbase = s.col_pbase;
  a.col_pfirst = s.col_pfirst;
  a.part_col = s.part_col;
  a.part_srank = s.part_srank;
  a.n_parts = s.n_parts;
  a.hist_st = s.hist_st;
  a.hist_go = s.hist_go;
  a.gk = std::max(s.gk, 1);
  a.acc_save = s.acc_save;
  a.gath = s.d_gath;
  a.gdone = s.d_gdone;
  a.tile_slots = s.tile_slots;
  a.row_base = s.row_base;
  a.deg = s.deg;
  a.idx = s.idx;
  a.syn = s.syn;
  a.wfx = s.wfx;
  a.v = s.v;
  a.ca = s.ca;
  a.na = s.na;
  a.ref = s.ref;
  a.hist_cnt = s.hist_cnt;
  a.hist_ids = s.hist_ids;
  a.ring = s.ring;
  a.net_cnt = s.net_cnt;
  a.col_spk = s.col_spk;
  if (s.rec_on) {
    a.rec_vprev = s.rec_vprev;
    a.rec_caprev = s.rec_caprev;
    a.rec_vt = s.rec_vt;
    a.rec_flags = s.rec_flags;
    a.rec_base = s.rec_base;
  }
  if (s.cfg.stdp) {
    a.syn_rw = s.syn;
    a.sp_y = s.sp_y;
    a.sp_x = s.sp_x;
    a.rev_ptr = s.rev_ptr;
    a.rev = s.rev;
    a.sp_pp = (float)exp(-s.cfg.dt / s.cfg.stdp_tau_plus);
    a.sp_pm = (float)exp(-s.cfg.dt / s.cfg.stdp_tau_minus);
    a.sp_ap = (float)s.cfg.stdp_a_plus;
    a.sp_am = (float)s.cfg.stdp_a_minus;
    a.sp_qmax = (int32_t)rint(s.cfg.stdp_w_max * 16384.0);
  }
  a.k = s.nk;
  return a;
}

// Allow each tile kernel the dynamic LDS that its static LDS leaves of the 160 KB of a
// workgroup, and record the largest static size.
template <int BLOCK>
hipError_t allow_large_lds() {
  const void* const fns[] = {(const void*)k_step_tile<BLOCK, true, kModelLif, false>,
                             (const void*)k_step_tile<BLOCK, false, kModelLif, false>,
                             (const void*)k_step_tile<BLOCK, false, kModelLifNa, false>,
                             (const void*)k_step_tile<BLOCK, false, kModelIzh, false>,
                             (const void*)k_step_tile<BLOCK, false, kModelLif, true>,
                             (const void*)k_step_tile<BLOCK, false, kModelLifNa, true>,
                             (const void*)k_step_tile<BLOCK, false, kModelIzh, true>};
  for (const void* f : fns) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, f);
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes >= kMaxLds) return hipErrorInvalidValue;
    g_tile_static_lds = std::max(g_tile_static_lds, (size_t)attr.sharedSizeBytes);
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kMaxLds - attr.sharedSizeBytes));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Allow the tile kernels the dynamic LDS beyond 64 KB (gfx950: 160 KB per workgroup).
hipError_t prepare_step_kernels() {
  hipError_t e;
  if ((e = allow_large_lds<64>()) != hipSuccess) return e;
  if ((e = allow_large_lds<128>()) != hipSuccess) return e;
  if ((e = allow_large_lds<256>()) != hipSuccess) return e;
  if ((e = allow_large_lds<512>()) != hipSuccess) return e;
  return allow_large_lds<1024>();
}

hipError_t launch_step(sim& s, int64_t u, int32_t delivery, int32_t block, int part) {
  switch (block) {
    case 64: return launch_step_b<64>(s, u, delivery, part);
    case 128: return launch_step_b<128>(s, u, delivery, part);
    case 256: return launch_step_b<256>(s, u, delivery, part);
    case 512: return launch_step_b<512>(s, u, delivery, part);
    case 1024: return launch_step_b<1024>(s, u, delivery, part);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_state(const sim& s) {
  const StepArgs a = make_step_args(s);
  const int64_t nall = s.n_neurons;
  int64_t blocks = (nall + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)blocks), dim3(256), 0, s.stream, a, s.model);
  return hipGetLastError();
}

}  // namespace dpsnn
