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
// neuron, its plastic synapses as 64-bit words (record index | delay - 1 | source id).  A
// postsynaptic spike then reads its ~1000 words contiguously and updates the records it names
// in place; the records of one step's spikes are distinct (one target each), so no two lanes
// touch the same record and no atomics are needed.
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

// Potentiation after the update of step u: one workgroup per column, each wave one of the
// column's spikes of step u at a time, its lanes over the spiking neuron's index words.
__global__ __launch_bounds__(256) void k_stdp_post(StepArgs a, int64_t u_arg) {
  const int64_t u = u_arg + (a.now_dev ? *a.now_dev : 0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t slot = u % a.dh;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  for (int32_t g = blockIdx.x; g < a.n_cols; g += gridDim.x) {
    const int64_t hb = slot * a.n_cols + g;
    const int32_t cnt = a.hist_cnt[hb];
    for (int32_t pos = wave; pos < cnt; pos += 4) {
      const int64_t j = (int64_t)g * a.npc + a.hist_ids[hb * a.npc + pos];
      const int64_t e1 = a.rev_ptr[j + 1];
      for (int64_t e = a.rev_ptr[j] + lane; e < e1; e += 64) {
        const uint64_t r = a.rev[e];
        const int64_t t = u - (int64_t)((r >> 35) & 31u) - 1;
        if (t < 0) continue;
        const float x = a.sp_x[(t % a.dh) * nall + (int64_t)(r >> 40)];
        const float t1 = a.sp_ap * x;
        const int32_t dq = (int32_t)__builtin_rintf(t1 * 16384.0f);
        if (dq == 0) continue;
        uint32_t* rec = a.syn_rw + (r & kRevRecMask);
        const uint32_t old = *rec;
        const int32_t w = min(rec_wq(old) + dq, a.sp_qmax);
        *rec = (old & 0xffffu) | ((uint32_t)w << 16);
      }
    }
  }
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

hipError_t launch_stdp_post(const sim& s, const StepArgs& a, int64_t u) {
  hipLaunchKernelGGL(k_stdp_post, dim3((unsigned)s.n_cols), dim3(256), 0, s.stream, a, u);
  return hipGetLastError();
}

}  // namespace dpsnn
