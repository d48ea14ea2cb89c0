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

// The neuron update and spike compaction of one column, shared by both strategies.
// in_of(k) returns the recurrent int32 input of local neuron k at step u.
template <int BLOCK, typename InputFn>
__device__ __forceinline__ void update_column(const StepArgs& a, int32_t g, int64_t u,
                                              const uint64_t* ptab, InputFn in_of, int32_t* wcnt,
                                              unsigned long long* red) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = lanemask_lt(lane);
  const int32_t net = a.col_net[g];
  const uint32_t key0 = a.net_key[2 * net], key1 = a.net_key[2 * net + 1];
  const uint32_t nl0 = (uint32_t)(a.col_local[g] * a.npc);
  const int32_t slot = (int32_t)(u % a.dh);
  uint16_t* out_ids = a.hist_ids + ((int64_t)slot * a.n_cols + g) * a.npc;
  int32_t running = 0;
  unsigned long long my_ext = 0, my_rec = 0;
  for (int k0 = 0; k0 < a.npc; k0 += BLOCK) {
    const int k = k0 + (int)threadIdx.x;
    bool spike = false;
    if (k < a.npc) {
      const int64_t j = (int64_t)g * a.npc + k;
      const Rand4 r = philox10(nl0 + (uint32_t)k, (uint32_t)u, 0u, kStreamExt, key0, key1);
      const int32_t n_ext = poisson_count(ptab, r.x);
      const uint32_t asum = (uint32_t)in_of(k) + (uint32_t)n_ext * (uint32_t)a.k.jfx;
      const float cur = (float)(int32_t)asum * 0x1p-16f;
      const float vprev = a.v[j];
      const float caprev = a.ca[j];
      int32_t rf = a.ref[j];
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
          spike = true;
          vnew = a.k.vreset;
          rf = a.k.tref;
        } else {
          vnew = vt;
        }
      }
      const float decayed = a.k.pc * caprev;
      const float canew = decayed + (spike ? a.k.alpha : 0.0f);
      a.v[j] = vnew;
      a.ca[j] = canew;
      a.ref[j] = (uint8_t)rf;
      my_ext += (unsigned long long)n_ext;
      if (spike) my_rec += (unsigned long long)(a.row_base[j + 1] - a.row_base[j]);
      if (a.rec_vprev) {
        const int64_t o = (u - a.rec_base) * (int64_t)a.n_cols * a.npc + j;
        a.rec_vprev[o] = vprev;
        a.rec_caprev[o] = caprev;
        a.rec_vt[o] = vt;
        a.rec_flags[o] = (uint8_t)((spike ? 1 : 0) | (refr ? 2 : 0));
      }
    }
    const unsigned long long m = __ballot(spike);
    if (lane == 0) wcnt[wave] = __popcll(m);
    __syncthreads();
    int32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int32_t c = wcnt[w];
      if (w < wave) before += c;
      tot += c;
    }
    if (spike) out_ids[running + before + __popcll(m & lt)] = (uint16_t)k;
    running += tot;
    __syncthreads();
  }
  const unsigned long long ext_all = block_sum_u64<BLOCK>(my_ext, red);
  const unsigned long long rec_all = block_sum_u64<BLOCK>(my_rec, red);
  if (threadIdx.x == 0) {
    a.hist_cnt[(int64_t)slot * a.n_cols + g] = running;
    atomicAdd(&a.net_cnt[4 * net + 0], (unsigned long long)running);
    atomicAdd(&a.net_cnt[4 * net + 1], rec_all);
    atomicAdd(&a.net_cnt[4 * net + 2], ext_all);
  }
}

template <int BLOCK>
__device__ __forceinline__ void load_ptab(const StepArgs& a, int32_t g, uint64_t* ptab) {
  const int32_t net = a.col_net[g];
  for (int q = threadIdx.x; q < kPoissonEntries; q += BLOCK)
    ptab[q] = a.net_ptab[(int64_t)net * kPoissonEntries + q];
}

// ---- ARRIVAL: gather + update, one workgroup per target column ------------------------
template <int BLOCK, bool TRAIN>
__global__ __launch_bounds__(BLOCK) void k_step_arrival(StepArgs a, int64_t u) {
  extern __shared__ int32_t acc[];
  __shared__ uint64_t ptab[kPoissonEntries];
  __shared__ int32_t it_pref[kMaxItems + 1];
  __shared__ int32_t it_hist[kMaxItems];
  __shared__ int32_t it_nbase[kMaxItems];
  __shared__ int32_t it_segc[kMaxItems];
  __shared__ int64_t cs_start[BLOCK];
  __shared__ int32_t cs_pref[BLOCK + 1];
  __shared__ int32_t wsum[BLOCK / 64];
  __shared__ unsigned long long red[BLOCK / 64];
  const int tid = threadIdx.x;
  const int n_items = a.nd * kMaxNbr;
  for (int32_t g = blockIdx.x; g < a.n_cols; g += gridDim.x) {
    load_ptab<BLOCK>(a, g, ptab);
    for (int k = tid; k < a.npc; k += BLOCK) acc[k] = 0;
    // 1. spike lists to gather: item (delay index dd, source rank r)
    const int nn = a.col_nn[g];
    int32_t carry = 0;
    for (int b = 0; b < n_items; b += BLOCK) {
      const int it = b + tid;
      int32_t cnt = 0;
      if (it < n_items) {
        const int dd = it / kMaxNbr, r = it - dd * kMaxNbr;
        const int64_t t = u - (a.d_min + dd);
        if (r < nn && t >= 0) {
          const int32_t s = a.col_nbr[g * kMaxNbr + r];
          const int32_t rank = a.col_rank[g * kMaxNbr + r];
          const int32_t hb = (int32_t)(t % a.dh) * a.n_cols + s;
          cnt = a.hist_cnt[hb];
          it_hist[it] = hb * a.npc;
          it_nbase[it] = s * a.npc;
          it_segc[it] = dd * kMaxNbr + rank;
        }
      }
      int32_t tot;
      const int32_t ex = block_excl_scan<BLOCK>(cnt, &tot, wsum);
      if (it < n_items) it_pref[it] = carry + ex;
      carry += tot;
    }
    if (tid == 0) it_pref[n_items] = carry;
    __syncthreads();
    const int32_t total = carry;
    // 2. chunks of BLOCK spike segments: locate, then stream their synapses into LDS
    unsigned long long streamed = 0;
    for (int32_t base = 0; base < total; base += BLOCK) {
      const int32_t q = base + tid;
      int32_t len = 0;
      int64_t start = 0;
      if (q < total) {
        int lo = 0, hi = n_items;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (it_pref[mid] <= q) lo = mid;
          else hi = mid;
        }
        const int32_t ksrc = a.hist_ids[it_hist[lo] + (q - it_pref[lo])];
        const int64_t i = (int64_t)it_nbase[lo] + ksrc;
        const uint16_t* sg = a.seg + i * a.segw + it_segc[lo];
        const int32_t o = sg[0], e = sg[1];
        start = a.row_base[i] + o;
        len = e - o;
      }
      int32_t tl;
      const int32_t ex = block_excl_scan<BLOCK>(len, &tl, wsum);
      cs_start[tid] = start;
      cs_pref[tid] = ex;
      if (tid == 0) cs_pref[BLOCK] = tl;
      streamed += (unsigned long long)tl;
      __syncthreads();
      for (int32_t f = tid; f < tl; f += BLOCK) {
        int lo = 0, hi = BLOCK;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (cs_pref[mid] <= f) lo = mid;
          else hi = mid;
        }
        const int64_t addr = cs_start[lo] + (f - cs_pref[lo]);
        const uint32_t w = a.syn[addr];
        const int32_t val = TRAIN ? a.wfx[addr] : (((int32_t)w) >> 16) * 4;
        atomicAdd(&acc[w & 0xffffu], val);
      }
      __syncthreads();
    }
    if (tid == 0 && streamed) atomicAdd(&a.net_cnt[4 * a.col_net[g] + 3], streamed);
    // 3. neuron update + compaction
    update_column<BLOCK>(a, g, u, ptab, [&](int k) { return acc[k]; }, wsum, red);
    __syncthreads();
  }
}

// ---- PUSH: update from the ring, then scatter ----------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_update_push(StepArgs a, int64_t u) {
  __shared__ uint64_t ptab[kPoissonEntries];
  __shared__ int32_t wsum[BLOCK / 64];
  __shared__ unsigned long long red[BLOCK / 64];
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  int32_t* slot = a.ring + (u % a.dh) * nall;
  for (int32_t g = blockIdx.x; g < a.n_cols; g += gridDim.x) {
    load_ptab<BLOCK>(a, g, ptab);
    __syncthreads();
    int32_t* in = slot + (int64_t)g * a.npc;
    update_column<BLOCK>(a, g, u, ptab, [&](int k) {
      const int32_t x = in[k];
      in[k] = 0;
      return x;
    }, wsum, red);
    __syncthreads();
  }
}

template <int BLOCK, bool TRAIN>
__global__ __launch_bounds__(BLOCK) void k_deliver_push(StepArgs a, int64_t u) {
  constexpr int NW = BLOCK / 64;
  __shared__ uint16_t segrow[NW][kMaxItems + 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nseg = a.nd * kMaxNbr;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int32_t uslot = (int32_t)(u % a.dh);
  for (int32_t g = blockIdx.x; g < a.n_cols; g += gridDim.x) {
    const int32_t ns = a.hist_cnt[(int64_t)uslot * a.n_cols + g];
    const uint16_t* ids = a.hist_ids + ((int64_t)uslot * a.n_cols + g) * a.npc;
    for (int32_t q = wave; q < ns; q += NW) {
      const int64_t i = (int64_t)g * a.npc + ids[q];
      const uint16_t* sg = a.seg + i * a.segw;
      for (int e = lane; e <= nseg; e += 64) segrow[wave][e] = sg[e];
      __builtin_amdgcn_wave_barrier();
      const int32_t len = segrow[wave][nseg];
      const int64_t rb = a.row_base[i];
      if (lane == 0 && len) atomicAdd(&a.net_cnt[4 * a.col_net[g] + 3], (unsigned long long)len);
      for (int32_t f = lane; f < len; f += 64) {
        int lo = 0, hi = nseg;  // last segment with start <= f
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if ((int32_t)segrow[wave][mid] <= f) lo = mid;
          else hi = mid;
        }
        const int dd = lo / kMaxNbr, r = lo - dd * kMaxNbr;
        const int32_t tc = a.col_nbr[g * kMaxNbr + r];
        const uint32_t w = a.syn[rb + f];
        const int32_t val = TRAIN ? a.wfx[rb + f] : (((int32_t)w) >> 16) * 4;
        const int64_t slot = (u + a.d_min + dd) % a.dh;
        atomicAdd(&a.ring[slot * nall + (int64_t)tc * a.npc + (w & 0xffffu)], val);
      }
      __builtin_amdgcn_wave_barrier();
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

template <int BLOCK>
hipError_t launch_step_t(sim& s, int64_t u, int32_t delivery, int part) {
  const StepArgs a = make_step_args(s);
  const bool train = s.wfx != nullptr;
  const int grid = s.n_cols;
  if (delivery == DPSNN_DELIVERY_ARRIVAL) {
    if (part == 1) return hipSuccess;
    const size_t lds = sizeof(int32_t) * (size_t)s.npc;
    if (train)
      hipLaunchKernelGGL((k_step_arrival<BLOCK, true>), dim3(grid), dim3(BLOCK), lds, s.stream, a, u);
    else
      hipLaunchKernelGGL((k_step_arrival<BLOCK, false>), dim3(grid), dim3(BLOCK), lds, s.stream, a, u);
    return hipGetLastError();
  }
  if (part != 1) hipLaunchKernelGGL((k_update_push<BLOCK>), dim3(grid), dim3(BLOCK), 0, s.stream, a, u);
  if (part != 0) {
    if (train)
      hipLaunchKernelGGL((k_deliver_push<BLOCK, true>), dim3(grid), dim3(BLOCK), 0, s.stream, a, u);
    else
      hipLaunchKernelGGL((k_deliver_push<BLOCK, false>), dim3(grid), dim3(BLOCK), 0, s.stream, a, u);
  }
  return hipGetLastError();
}

}  // namespace

StepArgs make_step_args(const sim& s) {
  StepArgs a{};
  a.npc = s.npc;
  a.nd = s.nd;
  a.d_min = s.cfg.d_min;
  a.dh = s.dh;
  a.segw = s.segw;
  a.n_cols = s.n_cols;
  a.col_net = s.col_net;
  a.col_local = s.col_local;
  a.col_nbr = s.col_nbr;
  a.col_nn = s.col_nn;
  a.col_rank = s.col_rank;
  a.net_key = s.net_key;
  a.net_ptab = s.net_ptab;
  a.row_base = s.row_base;
  a.seg = s.seg;
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
    case 64: return launch_step_t<64>(s, u, delivery, part);
    case 128: return launch_step_t<128>(s, u, delivery, part);
    case 256: return launch_step_t<256>(s, u, delivery, part);
    case 512: return launch_step_t<512>(s, u, delivery, part);
    case 1024: return launch_step_t<1024>(s, u, delivery, part);
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
