// step.hip -- the per-1 ms step on gfx950.
//
// The paper's simulator is mixed time- and event-driven (section 1): every neuron is
// integrated every step, and synaptic work is proportional to the spikes.  One step u:
//   input    A_j = (recurrent input due at step u) + n_j(u) * J_ext   (int32, 2^-16 mV)
//            n_j(u) ~ Poisson(ext_syn * rate * dt) from Philox at counter (j, u, 0, EXT),
//            inverse CDF against 63 integer thresholds
//   neuron   refractory: count down, V = V_reset, input discarded;
//            else V~ = ((P_m V) - (gamma Ca)) + A 2^-16, spike if V~ >= theta, then
//            V = V_reset and the refractory counter is set; Ca = P_c Ca + alpha s
//            (LIF with calcium-driven AHP, section 2), float32, no contraction
//   spikes   ascending local ids per column (wave ballots + workgroup prefix)
//   delivery each synapse (delay d) of a spike at step u contributes at step u + d
//
// Two delivery strategies, bit-identical because the input is an integer sum:
//   ARRIVAL  one workgroup per target column.  At step u it gathers, from the spike
//            history of the 3x3 source columns, the (delay d, target column) segment of
//            every row whose neuron spiked at u - d, accumulates into LDS with integer
//            atomics, then updates its neurons -- one fused kernel, no ring in HBM.
//   PUSH     update kernel reading a delay ring ring[u % DH][j], then a delivery kernel
//            that scatters each spiking row into ring[(u + d) % DH][target] with
//            device-scope integer atomics.
#include "dpsnn_internal.h"

namespace dpsnn {
namespace {

constexpr int kMaxItems = kMaxDelay * kMaxNbr;

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

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
  int32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int32_t v = wsum[w];
    if (w < wave) before += v;
    all += v;
  }
  __syncthreads();
  *total = all;
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
  unsigned long long all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) all += red[w];
  __syncthreads();
  return all;
}

// Number of thresholds <= x (the thresholds are non-decreasing).
__device__ __forceinline__ int32_t poisson_count(const uint64_t* tab, uint32_t x) {
  int lo = 0, hi = kPoissonEntries;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (tab[mid] <= (uint64_t)x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---- the neuron update, shared by both strategies ------------------------------------------
//
// Each thread owns the neurons k = m * BLOCK + tid (m < NPT) of the column.  Their state
// and external Poisson counts are fetched into registers first (prefetch_neurons), so that
// the loads and the Philox draws overlap with the gather of the delivered input; then
// finish_update applies the step and compacts the spikes in ascending order with one
// workgroup barrier (wave ballots, counts per (m, wave) in LDS).
template <int NPT>
struct NeuronRegs {
  float v[NPT];
  float ca[NPT];
  int32_t ref[NPT];
  int32_t next[NPT];
};

template <int BLOCK, int NPT>
__device__ __forceinline__ void prefetch_neurons(const StepArgs& a, int32_t g, int64_t u,
                                                 const uint64_t* ptab, NeuronRegs<NPT>& r) {
  const int32_t net = a.col_net[g];
  const uint32_t key0 = a.net_key[2 * net], key1 = a.net_key[2 * net + 1];
  const uint32_t nl0 = (uint32_t)(a.col_local[g] * a.npc);
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int k = m * BLOCK + (int)threadIdx.x;
    r.v[m] = 0.0f;
    r.ca[m] = 0.0f;
    r.ref[m] = 0;
    r.next[m] = 0;
    if (k < a.npc) {
      const int64_t j = (int64_t)g * a.npc + k;
      r.v[m] = a.v[j];
      r.ca[m] = a.ca[j];
      r.ref[m] = a.ref[j];
    }
  }
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int k = m * BLOCK + (int)threadIdx.x;
    if (k < a.npc) {
      const Rand4 x = philox10(nl0 + (uint32_t)k, (uint32_t)u, 0u, kStreamExt, key0, key1);
      r.next[m] = poisson_count(ptab, x.x);
    }
  }
}

// in_of(k) returns the recurrent int32 input of local neuron k at step u.  extra is added
// to the synapse counter of the network (the gather's streamed synapses).
template <int BLOCK, int NPT, typename InputFn>
__device__ __forceinline__ void finish_update(const StepArgs& a, int32_t g, int64_t u,
                                              NeuronRegs<NPT>& r, InputFn in_of, int32_t* wcnt,
                                              unsigned long long* red,
                                              unsigned long long extra) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = lanemask_lt(lane);
  const int32_t net = a.col_net[g];
  const int32_t slot = (int32_t)(u % a.dh);
  uint16_t* out_ids = a.hist_ids + ((int64_t)slot * a.n_cols + g) * a.npc;
  unsigned long long my_ext = 0, my_rec = 0;
  bool sp[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int k = m * BLOCK + (int)threadIdx.x;
    sp[m] = false;
    if (k < a.npc) {
      const int64_t j = (int64_t)g * a.npc + k;
      const uint32_t asum = (uint32_t)in_of(k) + (uint32_t)r.next[m] * (uint32_t)a.k.jfx;
      const float cur = (float)(int32_t)asum * 0x1p-16f;
      const float vprev = r.v[m];
      const float caprev = r.ca[m];
      int32_t rf = r.ref[m];
      float vnew, vt = 0.0f;
      bool refr = false;
      if (rf > 0) {
        refr = true;
        rf -= 1;
        vnew = a.k.vreset;
      } else {
        const float leak = a.k.pm * vprev;
        const float ahp = a.k.gam * caprev;
        const float drop = leak - ahp;
        vt = drop + cur;
        if (vt >= a.k.theta) {
          sp[m] = true;
          vnew = a.k.vreset;
          rf = a.k.tref;
        } else {
          vnew = vt;
        }
      }
      const float decayed = a.k.pc * caprev;
      const float canew = decayed + (sp[m] ? a.k.alpha : 0.0f);
      a.v[j] = vnew;
      a.ca[j] = canew;
      a.ref[j] = (uint8_t)rf;
      my_ext += (unsigned long long)r.next[m];
      if (sp[m]) my_rec += (unsigned long long)(a.row_base[j + 1] - a.row_base[j]);
      if (a.rec_vprev) {
        const int64_t o = (u - a.rec_base) * (int64_t)a.n_cols * a.npc + j;
        a.rec_vprev[o] = vprev;
        a.rec_caprev[o] = caprev;
        a.rec_vt[o] = vt;
        a.rec_flags[o] = (uint8_t)((sp[m] ? 1 : 0) | (refr ? 2 : 0));
      }
    }
  }
  unsigned long long bal[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    bal[m] = __ballot(sp[m]);
    if (lane == 0) wcnt[m * NW + wave] = __popcll(bal[m]);
  }
  __syncthreads();
  int32_t running = 0;
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    int32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int32_t c = wcnt[m * NW + w];
      if (w < wave) before += c;
      tot += c;
    }
    if (sp[m]) out_ids[running + before + __popcll(bal[m] & lt)] = (uint16_t)(m * BLOCK + threadIdx.x);
    running += tot;
  }
  const unsigned long long ext_all = block_sum_u64<BLOCK>(my_ext, red);
  const unsigned long long rec_all = block_sum_u64<BLOCK>(my_rec, red);
  const unsigned long long str_all = block_sum_u64<BLOCK>(extra, red);
  if (threadIdx.x == 0) {
    a.hist_cnt[(int64_t)slot * a.n_cols + g] = running;
    atomicAdd(&a.net_cnt[4 * net + 0], (unsigned long long)running);
    atomicAdd(&a.net_cnt[4 * net + 1], rec_all);
    atomicAdd(&a.net_cnt[4 * net + 2], ext_all);
    if (str_all) atomicAdd(&a.net_cnt[4 * net + 3], str_all);
  }
}

template <int BLOCK>
__device__ __forceinline__ void load_ptab(const StepArgs& a, int32_t g, uint64_t* ptab) {
  const int32_t net = a.col_net[g];
  for (int q = threadIdx.x; q < kPoissonEntries; q += BLOCK)
    ptab[q] = a.net_ptab[(int64_t)net * kPoissonEntries + q];
}

// ---- ARRIVAL: gather + update, one workgroup per target column ------------------------
//
// Work list of column g at step u: "items" (source column r, delay index dd), each the
// spike list of source column col_nbr[g][r] at step u - d_min - dd; every spike i of an
// item contributes one segment: the synapses of group (i, dd) that target column g.  Items
// of the own column come first (long segments), then the 8 neighbours (short ones), so
// that neighbouring segments have similar lengths.  Each wave takes batches of 64
// consecutive segments: lane l locates segment l of the batch (binary search over the item
// prefix, one spike id, one 32-byte group header) and then walks it in 16-byte pieces
// (four synapses per load, kPiecesInFlight loads in flight), adding each synapse's
// efficacy into the column's LDS accumulator with integer atomics.
constexpr int kPiecesInFlight = 4;

template <bool TRAIN>
__device__ __forceinline__ void add_piece(const StepArgs& a, int32_t* acc, const uint32_t* w,
                                          const int32_t* v, int32_t valid) {
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (e < valid) atomicAdd(&acc[w[e] & 0xffffu], TRAIN ? v[e] : (((int32_t)w[e]) >> 16) * 4);
}

template <int BLOCK, int NPT, bool TRAIN>
__global__ __launch_bounds__(BLOCK) void k_step_arrival(StepArgs a, int64_t u) {
  constexpr int NW = BLOCK / 64;
  extern __shared__ int32_t acc[];
  __shared__ uint64_t ptab[kPoissonEntries];
  __shared__ int32_t it_pref[kMaxItems + 1];
  __shared__ int32_t it_hist[kMaxItems];
  __shared__ int32_t it_nbase[kMaxItems];
  __shared__ int32_t it_hdr[kMaxItems];
  __shared__ int32_t it_rank[kMaxItems];
  __shared__ int32_t wsum[NPT * NW];
  __shared__ unsigned long long red[NW];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int32_t b = blockIdx.x; b < a.grid; b += gridDim.x) {
    const int32_t g = a.col_order[b];
    if (g < 0) continue;
    load_ptab<BLOCK>(a, g, ptab);
    for (int k = tid; k < a.npc; k += BLOCK) acc[k] = 0;
    const int nn = a.col_nn[g];
    int own = 0;  // rank of the own column in g's ascending neighbour list
    for (int r = 0; r < nn; ++r)
      if (a.col_nbr[g * kMaxNbr + r] == g) own = r;
    const int n_items = nn * a.nd;
    // 1. items and their spike counts; item = ro * nd + dd, ro = 0 the own column
    int32_t carry = 0;
    for (int b = 0; b < n_items; b += BLOCK) {
      const int it = b + tid;
      int32_t cnt = 0;
      if (it < n_items) {
        const int ro = it / a.nd, dd = it - ro * a.nd;
        const int r = ro == 0 ? own : (ro <= own ? ro - 1 : ro);
        const int64_t t = u - (a.d_min + dd);
        if (t >= 0) {
          const int32_t sc = a.col_nbr[g * kMaxNbr + r];
          const int32_t hb = (int32_t)(t % a.dh) * a.n_cols + sc;
          cnt = a.hist_cnt[hb];
          it_hist[it] = hb * a.npc;
          it_nbase[it] = sc * a.npc;
          it_hdr[it] = dd;
          it_rank[it] = a.col_rank[g * kMaxNbr + r];
        }
      }
      int32_t tot;
      const int32_t ex = block_excl_scan<BLOCK>(cnt, &tot, wsum);
      if (it < n_items) it_pref[it] = carry + ex;
      carry += tot;
    }
    if (tid == 0) it_pref[n_items] = carry;
    __syncthreads();  // items, the Poisson table and the zeroed accumulator are ready
    NeuronRegs<NPT> nr;
    prefetch_neurons<BLOCK, NPT>(a, g, u, ptab, nr);
    const int32_t total = carry;
    unsigned long long streamed = 0;
    // 2. gather: waves take batches of 64 segments
    for (int32_t b0 = wave * 64; b0 < total; b0 += NW * 64) {
      const int32_t q = b0 + lane;
      int64_t st = 0;
      int32_t ln = 0;
      if (q < total) {
        int lo = 0, hi = n_items;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (it_pref[mid] <= q) lo = mid;
          else hi = mid;
        }
        const int32_t ksrc = a.hist_ids[it_hist[lo] + (q - it_pref[lo])];
        const int64_t i = (int64_t)it_nbase[lo] + ksrc;
        const GroupHdr* h = a.hdr + i * a.nd + it_hdr[lo];
        const int r = it_rank[lo];
        const int32_t e1 = h->end[r];
        const int32_t e0 = r ? (int32_t)h->end[r - 1] : 0;
        st = h->start + e0;
        ln = e1 - e0;
      }
      streamed += (unsigned long long)ln;
      for (int32_t off = 0; __ballot(off < ln) != 0; off += 4 * kPiecesInFlight) {
        uint32_t w[kPiecesInFlight][4];
        int32_t v[kPiecesInFlight][4];
#pragma unroll
        for (int p = 0; p < kPiecesInFlight; ++p) {
          const int32_t o = off + 4 * p;
          if (o < ln) {
            __builtin_memcpy(&w[p][0], a.syn + st + o, 16);
            if (TRAIN) __builtin_memcpy(&v[p][0], a.wfx + st + o, 16);
          }
        }
#pragma unroll
        for (int p = 0; p < kPiecesInFlight; ++p) {
          const int32_t o = off + 4 * p;
          if (o < ln) add_piece<TRAIN>(a, acc, w[p], v[p], ln - o);
        }
      }
    }
    __syncthreads();  // all arrivals accumulated
    // 3. neuron update + compaction
    finish_update<BLOCK, NPT>(a, g, u, nr, [&](int k) { return acc[k]; }, wsum, red, streamed);
    __syncthreads();
  }
}

// ---- PUSH: update from the ring, then scatter ----------------------------------------------
template <int BLOCK, int NPT>
__global__ __launch_bounds__(BLOCK) void k_update_push(StepArgs a, int64_t u) {
  constexpr int NW = BLOCK / 64;
  __shared__ uint64_t ptab[kPoissonEntries];
  __shared__ int32_t wsum[NPT * NW];
  __shared__ unsigned long long red[NW];
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  int32_t* slot = a.ring + (u % a.dh) * nall;
  for (int32_t b = blockIdx.x; b < a.grid; b += gridDim.x) {
    const int32_t g = a.col_order[b];
    if (g < 0) continue;
    load_ptab<BLOCK>(a, g, ptab);
    __syncthreads();
    NeuronRegs<NPT> nr;
    prefetch_neurons<BLOCK, NPT>(a, g, u, ptab, nr);
    int32_t* in = slot + (int64_t)g * a.npc;
    finish_update<BLOCK, NPT>(a, g, u, nr, [&](int k) {
      const int32_t x = in[k];
      in[k] = 0;
      return x;
    }, wsum, red, 0ull);
    __syncthreads();
  }
}

__device__ __forceinline__ int32_t syn_value(const StepArgs& a, uint32_t w, int64_t addr,
                                             bool train) {
  return train ? a.wfx[addr] : (((int32_t)w) >> 16) * 4;
}

// Segment (target-column rank) of position f inside a group.
__device__ __forceinline__ int rank_in_group(const GroupHdr& h, int32_t f) {
  int r = 0;
#pragma unroll
  for (int q = 0; q < kMaxNbr - 1; ++q) r += ((int32_t)h.end[q] <= f) ? 1 : 0;
  return r;
}

template <int BLOCK, bool TRAIN>
__global__ __launch_bounds__(BLOCK) void k_deliver_push(StepArgs a, int64_t u) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int32_t uslot = (int32_t)(u % a.dh);
  for (int32_t g = blockIdx.x; g < a.n_cols; g += gridDim.x) {
    const int32_t ns = a.hist_cnt[(int64_t)uslot * a.n_cols + g];
    const uint16_t* ids = a.hist_ids + ((int64_t)uslot * a.n_cols + g) * a.npc;
    for (int32_t q = wave; q < ns; q += NW) {
      const int64_t i = (int64_t)g * a.npc + ids[q];
      unsigned long long pushed = 0;
      for (int dd = 0; dd < a.nd; ++dd) {
        const GroupHdr h = a.hdr[i * a.nd + dd];
        const int32_t len = h.end[kMaxNbr - 1];
        const int64_t slot = (u + a.d_min + dd) % a.dh;
        pushed += (unsigned long long)len;
        for (int32_t f = lane; f < len; f += 64) {
          const int r = rank_in_group(h, f);
          const int32_t tc = a.col_nbr[g * kMaxNbr + r];
          const uint32_t w = a.syn[h.start + f];
          atomicAdd(&a.ring[slot * nall + (int64_t)tc * a.npc + (w & 0xffffu)],
                    syn_value(a, w, h.start + f, TRAIN));
        }
      }
      if (lane == 0 && pushed) atomicAdd(&a.net_cnt[4 * a.col_net[g] + 3], pushed);
    }
  }
}

// ---- state initialisation: V uniform on [0, V_reset) from Philox at (j, 0, 0, INIT) --------
__global__ void k_init_state(StepArgs a) {
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nall;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = (int32_t)(j / a.npc);
    const int32_t k = (int32_t)(j - (int64_t)g * a.npc);
    const int32_t net = a.col_net[g];
    const Rand4 r = philox10((uint32_t)(a.col_local[g] * a.npc + k), 0u, 0u, kStreamInit,
                             a.net_key[2 * net], a.net_key[2 * net + 1]);
    const float unit = (float)(r.x >> 8) * 0x1p-24f;
    a.v[j] = a.k.vreset * unit;
    a.ca[j] = 0.0f;
    a.ref[j] = 0;
  }
}

template <int BLOCK, int NPT>
hipError_t launch_step_t(sim& s, int64_t u, int32_t delivery, int part) {
  const StepArgs a = make_step_args(s);
  const bool train = s.wfx != nullptr;
  const int grid = a.grid;
  if (delivery == DPSNN_DELIVERY_ARRIVAL) {
    if (part == 1) return hipSuccess;
    const size_t lds = sizeof(int32_t) * (size_t)s.npc;
    if (train)
      hipLaunchKernelGGL((k_step_arrival<BLOCK, NPT, true>), dim3(grid), dim3(BLOCK), lds, s.stream, a, u);
    else
      hipLaunchKernelGGL((k_step_arrival<BLOCK, NPT, false>), dim3(grid), dim3(BLOCK), lds, s.stream, a, u);
    return hipGetLastError();
  }
  if (part != 1) hipLaunchKernelGGL((k_update_push<BLOCK, NPT>), dim3(grid), dim3(BLOCK), 0, s.stream, a, u);
  if (part != 0) {
    if (train)
      hipLaunchKernelGGL((k_deliver_push<BLOCK, true>), dim3(grid), dim3(BLOCK), 0, s.stream, a, u);
    else
      hipLaunchKernelGGL((k_deliver_push<BLOCK, false>), dim3(grid), dim3(BLOCK), 0, s.stream, a, u);
  }
  return hipGetLastError();
}

template <int BLOCK>
hipError_t launch_step_b(sim& s, int64_t u, int32_t delivery, int part) {
  const int npt = (s.npc + BLOCK - 1) / BLOCK;
  if (npt <= 1) return launch_step_t<BLOCK, 1>(s, u, delivery, part);
  if (npt <= 2) return launch_step_t<BLOCK, 2>(s, u, delivery, part);
  if (npt <= 4) return launch_step_t<BLOCK, 4>(s, u, delivery, part);
  if (npt <= 8) return launch_step_t<BLOCK, 8>(s, u, delivery, part);
  return hipErrorInvalidValue;
}

}  // namespace

StepArgs make_step_args(const sim& s) {
  StepArgs a{};
  a.npc = s.npc;
  a.nd = s.nd;
  a.d_min = s.cfg.d_min;
  a.dh = s.dh;
  a.n_cols = s.n_cols;
  a.col_net = s.col_net;
  a.col_local = s.col_local;
  a.col_nbr = s.col_nbr;
  a.col_nn = s.col_nn;
  a.col_rank = s.col_rank;
  a.col_order = s.xcd_order ? s.col_order : s.col_order_rm;
  a.grid = s.xcd_order ? s.grid_xcd : s.n_cols;
  a.net_key = s.net_key;
  a.net_ptab = s.net_ptab;
  a.row_base = s.row_base;
  a.hdr = s.hdr;
  a.syn = s.syn;
  a.wfx = s.wfx;
  a.v = s.v;
  a.ca = s.ca;
  a.ref = s.ref;
  a.hist_cnt = s.hist_cnt;
  a.hist_ids = s.hist_ids;
  a.ring = s.ring;
  a.net_cnt = s.net_cnt;
  a.k = s.nk;
  return a;
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
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)blocks), dim3(256), 0, s.stream, a);
  return hipGetLastError();
}

}  // namespace dpsnn
