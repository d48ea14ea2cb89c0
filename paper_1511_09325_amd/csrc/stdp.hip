// stdp.hip -- spike-timing-dependent plasticity (sections 1-2 list it among the simulator's
// features; its measurements run with it off and no rule is printed).
//
// The rule is the all-to-all pair rule with exponential traces on the synapses of weight >= 0
// (the excitatory ones; inhibitory weights are negative and stay fixed), in int16 weight codes
// of 2^-14 mV bounded to [0, w_max]:
//   * at arrival (step u = emission + delay), after the spike has delivered the weight it
//     found, the weight drops by rint(a_minus * y-(j) * 2^14), y-(j) = P- y(j) the target's
//     trace of its spikes before u (the tile kernel does this while it gathers);
//   * after the update of step u, every plastic synapse (i, d) into a neuron j that spiked at
//     u rises by rint(a_plus * x_{u-d}(i) * 2^14), x_t(i) = P+ x_{t-1}(i) + s_i(t) the
//     source's trace: its spikes up to u - d, i.e. its arrivals at j up to u (this file).
// So each (arrival, postsynaptic spike) pair changes the weight once, by +a_plus
// exp(-(t_post - t_arr)/tau_plus) or -a_minus exp(-(t_arr - t_post)/tau_minus).
//
// The potentiation needs the synapses into a neuron.  The store is kept by source (rows split
// into parts by target tile), so a reverse index is built once at creation: per target
// neuron, its plastic synapses as 64-bit words (record index | delay - 1 | source id), sorted
// by source, so that the lanes reading one target's sources read neighbouring traces (a
// target's sources lie in a few columns).  A postsynaptic spike then reads its ~1000 words
// contiguously and updates the records they name in place; the records of one step's spikes
// are distinct (one target each), so no two lanes touch the same record and no atomics are
// needed.
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>

#include "dpsnn_internal.h"

namespace dpsnn {
namespace {

constexpr uint64_t kRevRecMask = (1ull << 35) - 1;

// One wave per source neuron: its plastic records (rank < 9, weight >= 0), counted per target
// or written to the target's range of the index.
template <bool FILL>
__global__ __launch_bounds__(256) void k_rev_pass(StepArgs a, int32_t* cnt,
                                                  unsigned long long* fill, uint64_t* rev) {
  const int lane = threadIdx.x & 63;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < nall; i += waves) {
    const int32_t g = (int32_t)(i / a.npc);
    const int32_t k = (int32_t)(i - (int64_t)g * a.npc);
    for (int p = 0; p < a.col_np[g]; ++p) {
      const uint8_t* ent = idx_entry(a, g, k, p);
      const int64_t st = ent_start(ent);
      const uint16_t* go = ent_goff(ent);
      const int32_t* pcol = a.part_col + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
      for (int dd = 0; dd < a.nd; ++dd) {
        for (int32_t f = go[dd] + lane; f < go[dd + 1]; f += 64) {
          const uint32_t w = a.syn[st + f];
          if (rec_rank(w) >= (uint32_t)kMaxPartCols || rec_wq(w) < 0) continue;
          const int64_t j = (int64_t)pcol[rec_rank(w)] * a.npc + rec_k(w);
          if (!FILL) {
            atomicAdd(&cnt[j], 1);
          } else {
            const unsigned long long pos = atomicAdd(&fill[j], 1ull);
            rev[pos] = (uint64_t)(st + f) | ((uint64_t)(a.d_min + dd - 1) << 35) |
                       ((uint64_t)i << 40);
          }
        }
      }
    }
  }
}

// Potentiation after the update of step u.  The step's spikes are spread over the whole
// grid: every workgroup turns the per-column spike counts into a prefix in LDS, then its
// waves take work items in a fixed stride over the grid's waves, an item being a quarter
// of one spike's index words (item q: spike q / 4, located by binary search over the
// prefix).  A lane holds four words in flight: their traces are loaded together, then the
// records whose change is not zero are read and written back.  Bursting columns therefore do
// not serialise on one workgroup.
constexpr int kPostBlock = 256;
constexpr int kPostSplit = 4;
constexpr int kPostInFlight = 4;

__global__ __launch_bounds__(kPostBlock) void k_stdp_post(StepArgs a, int64_t u_arg) {
  extern __shared__ int32_t pref[];  // [n_cols + 1]
  __shared__ int32_t wsum[kPostBlock / 64];
  const int64_t u = u_arg + (a.now_dev ? *a.now_dev : 0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t slot = u % a.dh;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int32_t* cnt = a.hist_cnt + slot * a.n_cols;
  // exclusive prefix of the column counts
  int32_t carry = 0;
  for (int32_t c0 = 0; c0 < a.n_cols; c0 += kPostBlock) {
    const int32_t c = c0 + tid;
    const int32_t x = c < a.n_cols ? cnt[c] : 0;
    int32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int32_t before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (c < a.n_cols) pref[c] = before + incl - x;
    for (int w = 0; w < kPostBlock / 64; ++w) carry += wsum[w];
    __syncthreads();
  }
  if (tid == 0) pref[a.n_cols] = carry;
  __syncthreads();
  const int64_t items = (int64_t)carry * kPostSplit;
  const int64_t waves = (int64_t)gridDim.x * (kPostBlock / 64);
  for (int64_t it = (int64_t)blockIdx.x * (kPostBlock / 64) + wave; it < items; it += waves) {
    const int32_t q = (int32_t)(it / kPostSplit), part = (int32_t)(it - (int64_t)q * kPostSplit);
    int lo = 0, hi = a.n_cols;  // the column g with pref[g] <= q < pref[g + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= q) lo = mid;
      else hi = mid;
    }
    const int32_t g = lo, pos = q - pref[lo];
    const int64_t j = (int64_t)g * a.npc + a.hist_ids[(slot * a.n_cols + g) * a.npc + pos];
    const int64_t b0 = a.rev_ptr[j], len = a.rev_ptr[j + 1] - b0;
    const int64_t e_lo = b0 + len * part / kPostSplit, e1 = b0 + len * (part + 1) / kPostSplit;
    for (int64_t e0 = e_lo + lane; e0 < e1; e0 += 64 * kPostInFlight) {
      uint64_t r[kPostInFlight];
      bool ok[kPostInFlight];
#pragma unroll
      for (int k = 0; k < kPostInFlight; ++k) {
        const int64_t e = e0 + 64 * k;
        r[k] = e < e1 ? a.rev[e] : 0ull;
        const int64_t t = u - (int64_t)((r[k] >> 35) & 31u) - 1;
        ok[k] = e < e1 && t >= 0;
      }
      int32_t dq[kPostInFlight];
#pragma unroll
      for (int k = 0; k < kPostInFlight; ++k) {
        float x = 0.0f;
        if (ok[k]) {
          const int64_t t = u - (int64_t)((r[k] >> 35) & 31u) - 1;
          x = a.sp_x[(t % a.dh) * nall + (int64_t)(r[k] >> 40)];
        }
        const float t1 = a.sp_ap * x;
        dq[k] = ok[k] ? (int32_t)__builtin_rintf(t1 * 16384.0f) : 0;
      }
      // the records whose weight changes (a source that spiked recently): read, then written
      uint32_t old[kPostInFlight];
#pragma unroll
      for (int k = 0; k < kPostInFlight; ++k) old[k] = dq[k] != 0 ? a.syn_rw[r[k] & kRevRecMask] : 0u;
#pragma unroll
      for (int k = 0; k < kPostInFlight; ++k) {
        if (dq[k] != 0) {
          const int32_t w = min(rec_wq(old[k]) + dq[k], a.sp_qmax);
          a.syn_rw[r[k] & kRevRecMask] = (old[k] & 0xffffu) | ((uint32_t)w << 16);
        }
      }
    }
  }
}

// Offsets of the segments of targets [j0, j0 + n) relative to the first one's start.
__global__ void k_rev_offsets(const int64_t* rev_ptr, int64_t j0, int32_t n, int32_t* off) {
  const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t <= n) off[t] = (int32_t)(rev_ptr[j0 + t] - rev_ptr[j0]);
}

int64_t grid_waves(int64_t n) {
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  return blocks < 1 ? 1 : blocks;
}

}  // namespace

hipError_t launch_rev_count(const sim& s, int32_t* cnt) {
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_rev_pass<false>, dim3((unsigned)grid_waves(s.n_neurons)), dim3(256), 0,
                     s.stream, a, cnt, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_rev_fill(const sim& s, unsigned long long* fill) {
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_rev_pass<true>, dim3((unsigned)grid_waves(s.n_neurons)), dim3(256), 0,
                     s.stream, a, nullptr, fill, s.rev);
  return hipGetLastError();
}

// The grid: four workgroups per compute unit of an MI355X (or fewer for small networks).
hipError_t launch_stdp_post(const sim& s, const StepArgs& a, int64_t u) {
  const unsigned grid = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(s.n_cols * 4, 1));
  hipLaunchKernelGGL(k_stdp_post, dim3(grid), dim3(kPostBlock),
                     sizeof(int32_t) * ((size_t)s.n_cols + 1), s.stream, a, u);
  return hipGetLastError();
}

// Sort every target's index words by source (bits 40-63), in chunks of whole targets of at
// most `chunk` words: a segmented radix sort per chunk through a buffer of that size.  Order
// within a target does not change results, only which traces neighbouring lanes read.
hipError_t sort_rev(const sim& s, int64_t chunk, int32_t max_segs, uint64_t* alt, int32_t* off,
                    void* temp, size_t temp_bytes, const std::vector<int64_t>& h_ptr) {
  const int64_t N = s.n_neurons;
  int64_t j0 = 0;
  while (j0 < N) {
    int64_t j1 = j0;
    while (j1 < N && j1 - j0 < max_segs && h_ptr[(size_t)j1 + 1] - h_ptr[(size_t)j0] <= chunk) ++j1;
    if (j1 == j0) return hipErrorInvalidValue;  // a target with more words than a chunk
    const int32_t nseg = (int32_t)(j1 - j0);
    const int64_t items = h_ptr[(size_t)j1] - h_ptr[(size_t)j0];
    hipLaunchKernelGGL(k_rev_offsets, dim3((unsigned)((nseg + 256) / 256)), dim3(256), 0, s.stream,
                       s.rev_ptr, j0, nseg, off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* keys = s.rev + h_ptr[(size_t)j0];
    rocprim::double_buffer<uint64_t> db(keys, alt);
    size_t tb = temp_bytes;
    e = rocprim::segmented_radix_sort_keys(temp, tb, db, (unsigned int)items, (unsigned int)nseg,
                                           off, off + 1, 40, 64, s.stream);
    if (e != hipSuccess) return e;
    if (db.current() != keys) {
      e = hipMemcpyAsync(keys, db.current(), sizeof(uint64_t) * (size_t)items,
                         hipMemcpyDeviceToDevice, s.stream);
      if (e != hipSuccess) return e;
    }
    j0 = j1;
  }
  return hipSuccess;
}

// Temporary storage the sort needs for chunks of at most `chunk` words and `segs` segments.
hipError_t sort_rev_temp_bytes(int64_t chunk, int32_t segs, size_t* bytes) {
  rocprim::double_buffer<uint64_t> db(nullptr, nullptr);
  *bytes = 0;
  return rocprim::segmented_radix_sort_keys(nullptr, *bytes, db, (unsigned int)chunk,
                                            (unsigned int)segs, (int32_t*)nullptr,
                                            (int32_t*)nullptr + 1, 40, 64, (hipStream_t)0);
}

}  // namespace dpsnn
