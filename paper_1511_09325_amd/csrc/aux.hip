// aux.hip -- raster recording, the pending-input view, synapse export, weight quantiser.
#include "dpsnn_internal.h"

namespace dpsnn {
namespace {

// Raster: exclusive scan of this step's per-column spike counts (one workgroup), giving
// each column its place in the ascending global id list of the step.
__global__ __launch_bounds__(1024) void k_raster_scan(const int32_t* hist_cnt, int32_t n_cols,
                                                      int32_t dh, int64_t u_arg,
                                                      const int64_t* now_dev, int64_t* ras_off,
                                                      int64_t* colofs, int64_t cap,
                                                      int32_t* flags) {
  __shared__ int64_t wsum[16];
  const int64_t u = u_arg + (now_dev ? *now_dev : 0);
  const int32_t slot = (int32_t)(u % dh);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t carry = ras_off[u];
  for (int32_t b = 0; b < n_cols; b += 1024) {
    const int32_t g = b + threadIdx.x;
    const int64_t x = g < n_cols ? hist_cnt[(int64_t)slot * n_cols + g] : 0;
    int64_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wave) before += wsum[w];
      all += wsum[w];
    }
    __syncthreads();
    if (g < n_cols) colofs[g] = carry + before + incl - x;
    carry += all;
  }
  if (threadIdx.x == 0) {
    ras_off[u + 1] = carry;
    if (carry > cap) flags[0] = 1;
  }
}

__global__ __launch_bounds__(256) void k_raster_copy(const int32_t* hist_cnt,
                                                     const uint16_t* hist_ids, int32_t n_cols,
                                                     int32_t npc, int32_t dh, int64_t u_arg,
                                                     const int64_t* now_dev,
                                                     const int64_t* colofs, int32_t* ras_ids,
                                                     int64_t cap) {
  const int32_t g = blockIdx.x;
  const int64_t u = u_arg + (now_dev ? *now_dev : 0);
  const int32_t slot = (int32_t)(u % dh);
  const int32_t n = hist_cnt[(int64_t)slot * n_cols + g];
  const int64_t base = colofs[g];
  if (base + n > cap) return;
  const uint16_t* ids = hist_ids + ((int64_t)slot * n_cols + g) * npc;
  for (int32_t q = threadIdx.x; q < n; q += 256) ras_ids[base + q] = g * npc + ids[q];
}

// Pending-input view of the arrival strategy: pend[q][j] = sum over spikes of steps
// t in [now - d_max, now) and synapses of delay d with t + d = now + q, restricted to the
// target columns [g0, g1) of one network (j relative to column g0).
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_pend_arrival(StepArgs a, int64_t now, int32_t* pend,
                                                      int32_t g0, int32_t g1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n_net = (int64_t)(g1 - g0) * a.npc;
  const int32_t g = g0 + blockIdx.x;  // source columns of the same network
  const int d_max = a.d_min + a.nd - 1;
  for (int back = 1; back <= d_max; ++back) {
    const int64_t t = now - back;
    if (t < 0) break;
    const int32_t slot = (int32_t)(t % a.dh);
    const int32_t ns = a.hist_cnt[(int64_t)slot * a.n_cols + g];
    const uint16_t* ids = a.hist_ids + ((int64_t)slot * a.n_cols + g) * a.npc;
    const int np = a.col_np[g];
    for (int32_t q = wave; q < ns; q += 4) {
      for (int p = 0; p < np; ++p) {
        const uint8_t* ent = idx_entry(a, g, ids[q], p);
        const int64_t st = ent_start(ent);
        const uint16_t* go = ent_goff(ent);
        const int32_t* pcol = a.part_col + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
        for (int dd = 0; dd < a.nd; ++dd) {
          const int64_t due = t + a.d_min + dd;
          if (due < now) continue;
          for (int32_t f = go[dd] + lane; f < go[dd + 1]; f += 64) {
            const uint32_t w = a.syn[st + f];
            if (rec_rank(w) == (uint32_t)kDummyRank) continue;
            const int32_t tc = pcol[rec_rank(w)];
            const int32_t val = TRAIN ? a.wfx[st + f] : rec_w32(w);
            atomicAdd(&pend[(due - now) * n_net + (int64_t)(tc - g0) * a.npc + rec_k(w)], val);
          }
        }
      }
    }
  }
}

// Export rows [i0, i1) (global neuron ids) in device order with network-local targets, the
// padding marked with delay 0 (the host drops it and sorts each row into canonical order).
__global__ __launch_bounds__(256) void k_export_rows(StepArgs a, int32_t g0, int64_t i0,
                                                     int64_t i1, const int64_t* out_off,
                                                     int32_t* tgt, uint8_t* dly, int16_t* wq) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t i = i0 + (int64_t)blockIdx.x * 4 + wave; i < i1; i += (int64_t)gridDim.x * 4) {
    const int32_t g = (int32_t)(i / a.npc);
    const int32_t k = (int32_t)(i - (int64_t)g * a.npc);
    const int64_t ob = out_off[i - i0];
    const int64_t rb = a.row_base[i];
    for (int p = 0; p < a.col_np[g]; ++p) {
      const uint8_t* ent = idx_entry(a, g, k, p);
      const int64_t st = ent_start(ent);
      const uint16_t* go = ent_goff(ent);
      const int32_t* pcol = a.part_col + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
      for (int dd = 0; dd < a.nd; ++dd) {
        for (int32_t f = go[dd] + lane; f < go[dd + 1]; f += 64) {
          const uint32_t w = a.syn[st + f];
          const int64_t o = ob + (st - rb) + f;
          if (rec_rank(w) == (uint32_t)kDummyRank) {
            tgt[o] = -1;
            dly[o] = 0;
            wq[o] = 0;
            continue;
          }
          const int32_t tc = pcol[rec_rank(w)];
          tgt[o] = (tc - g0) * a.npc + (int32_t)rec_k(w);
          dly[o] = (uint8_t)(a.d_min + dd);
          wq[o] = (int16_t)(w >> 16);
        }
      }
    }
  }
}

// Spike-history entries of every spike held in the history (after a restore).
__global__ __launch_bounds__(256) void k_fill_entries(StepArgs a) {
  const int32_t g = blockIdx.x, slot = blockIdx.y;
  const int32_t ns = a.hist_cnt[(int64_t)slot * a.n_cols + g];
  const uint16_t* ids = a.hist_ids + ((int64_t)slot * a.n_cols + g) * a.npc;
  for (int32_t q = threadIdx.x; q < ns; q += 256) write_entries(a, g, ids[q], slot, q);
}

__global__ void k_set_now(int64_t* d_now, int64_t now) { *d_now = now; }
__global__ void k_zero_u64(uint64_t* p) { *p = 0; }

// splitmix64 finaliser (Steele, Lea, Flood 2014), used to mix state words into a digest
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Order-independent digest of the dynamic state: V, Ca, refractory counters and the spike
// history of the last DH steps (which determines every pending input); with plasticity also
// the traces and the n_rec records of the store (the weights).
__global__ __launch_bounds__(256) void k_digest(StepArgs a, int64_t now, int64_t n_rec,
                                                uint64_t* out) {
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  uint64_t h = 0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n_rec; r += (int64_t)gridDim.x * 256)
    h += mix64(((uint64_t)r << 32) ^ a.syn[r] ^ 0xD6E8FEB86659FD93ull);
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < nall; j += (int64_t)gridDim.x * 256) {
    if (a.sp_y) {
      h += mix64(((uint64_t)__float_as_uint(a.sp_y[j]) << 32) ^ (uint64_t)j ^ 0xA0761D6478BD642Full);
      for (int q = 0; q < a.dh; ++q)
        h += mix64(((uint64_t)__float_as_uint(a.sp_x[(int64_t)q * nall + j]) << 32) ^
                   ((uint64_t)j << 6) ^ (uint64_t)q ^ 0xE7037ED1A0B428DBull);
    }
    const uint64_t v = __float_as_uint(a.v[j]), c = __float_as_uint(a.ca[j]);
    const uint64_t na = a.na ? __float_as_uint(a.na[j]) : 0u;  // sodium AHP variable, if kept
    h += mix64(((uint64_t)j << 2) ^ (v << 32) ^ c ^ ((uint64_t)a.ref[j] << 40) ^ (na << 7));
    const int32_t g = (int32_t)(j / a.npc), k = (int32_t)(j - (int64_t)g * a.npc);
    for (int back = 1; back <= a.dh - 1; ++back) {
      const int64_t t = now - back;
      if (t < 0) break;
      const int64_t hb = (t % a.dh) * a.n_cols + g;
      if (k < a.hist_cnt[hb])
        h += mix64(0x9E3779B97F4A7C15ull * (uint64_t)(t + 1) ^ ((uint64_t)g << 20) ^
                   a.hist_ids[hb * a.npc + k] ^ ((uint64_t)k << 48));
    }
  }
  for (int off = 32; off > 0; off >>= 1) h += __shfl_down(h, off);
  if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long*)out, (unsigned long long)h);
}

// Train mode: int32 efficacies rint(w * 2^16) from the float32 master weights (mV).
__global__ void k_quantise(const float* w, int32_t* wfx, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    wfx[e] = (int32_t)__builtin_rintf(w[e] * 65536.0f);
}

// One network's share of the recorded raster: per step t0 + i the range of its ids [lo, hi)
// within the step's ascending global ids, by binary search (one thread per step).
__global__ __launch_bounds__(256) void k_raster_bounds(const int64_t* ras_off,
                                                       const int32_t* ras_ids, int64_t t0,
                                                       int64_t nsteps, int32_t lo, int32_t hi,
                                                       int64_t* bounds) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsteps) return;
  const int64_t a = ras_off[t0 + i], b = ras_off[t0 + i + 1];
  int64_t x = a, n = b - a;  // first id >= lo
  while (n > 0) {
    const int64_t h = n >> 1;
    if (ras_ids[x + h] < lo) { x += h + 1; n -= h + 1; } else n = h;
  }
  int64_t y = x, m = b - x;  // first id >= hi
  while (m > 0) {
    const int64_t h = m >> 1;
    if (ras_ids[y + h] < hi) { y += h + 1; m -= h + 1; } else m = h;
  }
  bounds[2 * i] = x;
  bounds[2 * i + 1] = y;
}

// Gathers those ranges, made network-local (minus lo), into out at the steps' offsets
// (dst_off[i], exclusive prefix of the range lengths); ids past n are dropped.  One
// workgroup per step.
__global__ __launch_bounds__(256) void k_raster_take(const int32_t* ras_ids,
                                                     const int64_t* bounds,
                                                     const int64_t* dst_off, int32_t lo,
                                                     int64_t n, int32_t* out) {
  const int64_t i = blockIdx.x;
  const int64_t x = bounds[2 * i], y = bounds[2 * i + 1], d = dst_off[i];
  for (int64_t k = x + threadIdx.x; k < y; k += blockDim.x) {
    const int64_t o = d + (k - x);
    if (o < n) out[o] = ras_ids[k] - lo;
  }
}

// Length of each of those ranges: len[i] = bounds[2i + 1] - bounds[2i].
__global__ __launch_bounds__(256) void k_raster_lengths(const int64_t* bounds, int64_t nsteps,
                                                        int64_t* len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsteps) len[i] = bounds[2 * i + 1] - bounds[2 * i];
}

}  // namespace

// One network's spikes of steps [t0, t0 + nsteps) from the raster (synchronous): bounds
// receives the per-step ranges (device, 2 * nsteps), then, when out is given, the first n ids
// go to out (device) at the offsets dst_off (device, nsteps).
hipError_t launch_raster_bounds(const sim& s, int64_t t0, int64_t nsteps, int32_t lo, int32_t hi,
                                int64_t* bounds) {
  if (nsteps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_bounds, dim3((unsigned)((nsteps + 255) / 256)), dim3(256), 0,
                     s.stream, s.ras_off, s.ras_ids, t0, nsteps, lo, hi, bounds);
  return hipGetLastError();
}

hipError_t launch_raster_take(const sim& s, int64_t nsteps, const int64_t* bounds,
                              const int64_t* dst_off, int32_t lo, int64_t n, int32_t* out) {
  if (nsteps <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_take, dim3((unsigned)nsteps), dim3(256), 0, s.stream, s.ras_ids,
                     bounds, dst_off, lo, n, out);
  return hipGetLastError();
}

hipError_t launch_raster_lengths(const sim& s, int64_t nsteps, const int64_t* bounds,
                                 int64_t* len) {
  if (nsteps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_lengths, dim3((unsigned)((nsteps + 255) / 256)), dim3(256), 0,
                     s.stream, bounds, nsteps, len);
  return hipGetLastError();
}

hipError_t launch_raster(sim& s, int64_t u) {
  const int64_t* nd = s.graph_mode ? s.d_now : nullptr;
  hipLaunchKernelGGL(k_raster_scan, dim3(1), dim3(1024), 0, s.stream, s.hist_cnt, s.n_cols, s.dh,
                     u, nd, s.ras_off, s.ras_colofs, s.cfg.raster_capacity, s.flags);
  hipLaunchKernelGGL(k_raster_copy, dim3(s.n_cols), dim3(256), 0, s.stream, s.hist_cnt,
                     s.hist_ids, s.n_cols, s.npc, s.dh, u, nd, s.ras_colofs, s.ras_ids,
                     s.cfg.raster_capacity);
  return hipGetLastError();
}

hipError_t launch_fill_entries(const sim& s) {
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_fill_entries, dim3(s.n_cols, s.dh), dim3(256), 0, s.stream, a);
  return hipGetLastError();
}

hipError_t launch_set_now(const sim& s, int64_t now) {
  hipLaunchKernelGGL(k_set_now, dim3(1), dim3(1), 0, s.stream, s.d_now, now);
  return hipGetLastError();
}

hipError_t launch_digest(const sim& s, uint64_t* out) {
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s.stream, out);
  int64_t blocks = (s.n_neurons + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  const int64_t n_rec = s.cfg.stdp ? s.n_syn_padded : 0;
  hipLaunchKernelGGL(k_digest, dim3((unsigned)blocks), dim3(256), 0, s.stream, a, s.now, n_rec,
                     out);
  return hipGetLastError();
}

hipError_t launch_pend_view(const sim& s, int32_t* pend, int32_t g0, int32_t g1) {
  const StepArgs a = make_step_args(s);
  if (s.wfx)
    hipLaunchKernelGGL(k_pend_arrival<true>, dim3(g1 - g0), dim3(256), 0, s.stream, a, s.now,
                       pend, g0, g1);
  else
    hipLaunchKernelGGL(k_pend_arrival<false>, dim3(g1 - g0), dim3(256), 0, s.stream, a, s.now,
                       pend, g0, g1);
  return hipGetLastError();
}

hipError_t launch_export_rows(const sim& s, int32_t net, int64_t i0, int64_t i1, int32_t* tgt,
                              uint8_t* dly, int16_t* wq, const int64_t* out_off) {
  const StepArgs a = make_step_args(s);
  const int32_t g0 = s.net_col0[net];
  int64_t blocks = (i1 - i0 + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_export_rows, dim3((unsigned)blocks), dim3(256), 0, s.stream, a, g0, i0, i1,
                     out_off, tgt, dly, wq);
  return hipGetLastError();
}

hipError_t launch_quantise(const sim& s) {
  // the padded layout, dummies included (their master weight is 0)
  int64_t blocks = (s.n_syn_padded + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_quantise, dim3((unsigned)blocks), dim3(256), 0, s.stream, s.wf32, s.wfx,
                     s.n_syn_padded);
  return hipGetLastError();
}

}  // namespace dpsnn
