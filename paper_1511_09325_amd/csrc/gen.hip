// gen.hip -- network construction on the device.
//
// Follows the paper's network description (section 2, Methods): columns of point neurons,
// 80 % excitatory, each neuron connected to neurons of its own column with a fixed pair
// probability and to the neighbouring columns with a probability decaying with distance;
// plus the workload's integer delays and normal weights.  Every pair (i, j) of a source
// neuron i and a candidate target j in the torus stencil around i's column is one
// Bernoulli trial decided by Philox4x32-10 at counter (j, i, 0, SYN) of the network's key:
//   connected iff word x < threshold(column pair)       (threshold = floor(p 2^32))
//   delay      d = d_min + floor(word y * nd / 2^32)
//   weight     mu + sigma * z, z = (sum of 12 16-bit halves of words z, w and of the four
//              words at counter (j, i, 1, SYN) - 393210) / 65536, in double, no FMA,
//              quantised to int16 at 2^-14 mV with round-half-even.
// Each row is split into parts, one per tile of the native tiling that the source
// column's stencil touches (the part of each stencil rank is in col_part); a part holds
// one group per delay, each record carrying the rank of its target column inside the part
// (col_prank), targets
// in canonical order inside a group, and each group padded with dummy records to a
// multiple of 4 so that 16-byte words never straddle two groups.  Two passes over the
// candidates: the first counts each row's padded length and out-degree (then an exclusive
// scan over rows gives the row starts), the second counts again, lays the row out and
// fills it.
#include "dpsnn_internal.h"

namespace dpsnn {
namespace {

struct GenArgs {
  int32_t npc, n_exc, nd, d_min;
  int64_t row0, rows;
  const int32_t* col_net;
  const int32_t* col_local;
  const int32_t* col_nbr;
  const int32_t* col_nn;
  const int32_t* col_part;
  const int32_t* col_prank;
  const int32_t* col_np;
  const int64_t* col_pbase;
  const uint64_t* col_thr;
  const uint32_t* net_key;
  double we_mu, we_sigma, wi_mu, wi_sigma;
  int32_t* row_len;        // count pass output: padded row length
  int32_t* deg;            // count pass output: out-degree
  const int64_t* row_base; // fill pass input
  uint32_t* syn;           // fill pass output
  uint8_t* idx;            // fill pass output: row-index entries
  int32_t idxw;
};

// per-wave LDS of the construction kernels, for stencils of at most NBR distinct columns
// (rows per workgroup: WAVES, one wave each; fewer for the 7x7 stencil's larger tables)
template <int NBR>
struct RowLayout {
  int32_t cnt[kMaxDelay][NBR];            // synapses of (delay, stencil rank)
  int32_t seg[kMaxDelay][NBR];            // fill: first record of (delay, rank) in the row
  int32_t gst[kMaxParts][kMaxDelay + 1];  // fill: start of group (part, delay); [nd] = end
  int32_t pad[kMaxParts][kMaxDelay];      // fill: first padding record of group (part, delay)
};

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Decide one candidate: returns connected flag and delay index (0..nd-1).
__device__ __forceinline__ bool decide(const GenArgs& a, int64_t i, int64_t jglob, uint32_t jl,
                                       uint32_t il, uint32_t k0, uint32_t k1, uint64_t thr,
                                       bool valid, int& dd, Rand4& r) {
  r = philox10(jl, il, 0u, kStreamSyn, k0, k1);
  const bool conn = valid && (jglob != i) && ((uint64_t)r.x < thr);
  dd = (int)(((uint64_t)r.y * (uint64_t)a.nd) >> 32);
  return conn;
}

// Synapse counts of row i per (delay, rank) into L.cnt (one wave).
template <int NBR>
__device__ void count_row(const GenArgs& a, int64_t i, int32_t g, uint32_t il, uint32_t k0,
                          uint32_t k1, RowLayout<NBR>& L) {
  const int lane = threadIdx.x & 63;
  const int nn = a.col_nn[g];
  for (int q = lane; q < kMaxDelay * NBR; q += 64) (&L.cnt[0][0])[q] = 0;
  __builtin_amdgcn_wave_barrier();
  for (int r = 0; r < nn; ++r) {
    const int32_t tc = a.col_nbr[g * kMaxNbr + r];
    const uint64_t thr = a.col_thr[g * kMaxNbr + r];
    const uint32_t tl0 = (uint32_t)(a.col_local[tc] * a.npc);
    int32_t mine = 0;
    for (int kb = 0; kb < a.npc; kb += 64) {
      const int k = kb + lane;
      int dd;
      Rand4 rr4;
      const bool conn = decide(a, i, (int64_t)tc * a.npc + k, tl0 + (uint32_t)k, il, k0, k1,
                               thr, k < a.npc, dd, rr4);
      for (int q = 0; q < a.nd; ++q) {
        const unsigned long long m = __ballot(conn && dd == q);
        if (lane == q) mine += __popcll(m);
      }
    }
    if (lane < a.nd) L.cnt[lane][r] = mine;
  }
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int32_t padded(int32_t n) { return (n + 3) & ~3; }

template <int NBR, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gen_count(GenArgs a) {
  __shared__ RowLayout<NBR> lay[WAVES];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  RowLayout<NBR>& L = lay[wave];
  for (int64_t rr = (int64_t)blockIdx.x * WAVES + wave; rr < a.rows;
       rr += (int64_t)gridDim.x * WAVES) {
    const int64_t i = a.row0 + rr;
    const int32_t g = (int32_t)(i / a.npc);
    const int32_t kk = (int32_t)(i - (int64_t)g * a.npc);
    const int32_t net = a.col_net[g];
    const uint32_t il = (uint32_t)(a.col_local[g] * a.npc + kk);
    count_row(a, i, g, il, a.net_key[2 * net], a.net_key[2 * net + 1], L);
    const int nn = a.col_nn[g], np = a.col_np[g];
    // lane dd: padded length of every group (part, dd) and the out-degree of delay dd
    int32_t len = 0, used = 0;
    if (lane < a.nd) {
      for (int p = 0; p < np; ++p) {
        int32_t glen = 0;
        for (int r = 0; r < nn; ++r)
          if (a.col_part[g * kMaxNbr + r] == p) glen += L.cnt[lane][r];
        len += padded(glen);
        used += glen;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      len += __shfl_down(len, off);
      used += __shfl_down(used, off);
    }
    if (lane == 0) {
      a.row_len[i] = len;
      a.deg[i] = used;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int NBR, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gen_fill(GenArgs a) {
  __shared__ RowLayout<NBR> lay[WAVES];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = lanemask_lt(lane);
  RowLayout<NBR>& L = lay[wave];
  for (int64_t rr = (int64_t)blockIdx.x * WAVES + wave; rr < a.rows;
       rr += (int64_t)gridDim.x * WAVES) {
    const int64_t i = a.row0 + rr;
    const int32_t g = (int32_t)(i / a.npc);
    const int32_t kk = (int32_t)(i - (int64_t)g * a.npc);
    const int32_t net = a.col_net[g];
    const uint32_t il = (uint32_t)(a.col_local[g] * a.npc + kk);
    const uint32_t k0 = a.net_key[2 * net], k1 = a.net_key[2 * net + 1];
    count_row(a, i, g, il, k0, k1, L);
    const int nn = a.col_nn[g], np = a.col_np[g];
    // layout: parts in order, inside a part the groups by delay; lane dd owns delay dd
    int32_t base = 0;
    for (int p = 0; p < np; ++p) {
      int32_t glen = 0;
      if (lane < a.nd)
        for (int r = 0; r < nn; ++r)
          if (a.col_part[g * kMaxNbr + r] == p) glen += L.cnt[lane][r];
      const int32_t plen = lane < a.nd ? padded(glen) : 0;
      int32_t incl = plen;
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      if (lane < a.nd) {
        L.gst[p][lane] = base + incl - plen;
        L.pad[p][lane] = base + incl - plen + glen;
      }
      const int32_t tot = __shfl(incl, 63);
      if (lane == 0) L.gst[p][a.nd] = base + tot;
      base += tot;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < a.nd) {
      // segment (dd, r) follows the earlier ranks of the same part inside group (part, dd)
      for (int r = 0; r < nn; ++r) {
        const int p = a.col_part[g * kMaxNbr + r];
        int32_t at = L.gst[p][lane];
        for (int r2 = 0; r2 < r; ++r2)
          if (a.col_part[g * kMaxNbr + r2] == p) at += L.cnt[lane][r2];
        L.seg[lane][r] = at;
      }
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t rb = a.row_base[i];
    uint32_t* out = a.syn + rb;
    // row-index entries of the parts: start of the part, the start of each group, then the
    // number of the part's synapses (without the padding)
    for (int p = 0; p < np; ++p) {
      uint8_t* ent = a.idx + (a.col_pbase[g] + (int64_t)kk * np + p) * a.idxw;
      const int32_t p0 = L.gst[p][0];
      if (lane == 0) *(int64_t*)ent = rb + p0;
      for (int dd = lane; dd <= a.nd; dd += 64) ((uint16_t*)(ent + 8))[dd] = (uint16_t)(L.gst[p][dd] - p0);
      int32_t real = lane < a.nd ? L.pad[p][lane] - L.gst[p][lane] : 0;
      for (int off = 32; off > 0; off >>= 1) real += __shfl_down(real, off);
      if (lane == 0) ((uint16_t*)(ent + 8))[a.nd + 1] = (uint16_t)real;
    }
    // dummy records (rank 9, weight 0) in the padding at the end of each group
    for (int p = 0; p < np; ++p)
      for (int dd = 0; dd < a.nd; ++dd)
        for (int32_t q = L.pad[p][dd] + lane; q < L.gst[p][dd + 1]; q += 64) out[q] = kDummyRecord;
    const bool exc = kk < a.n_exc;
    const double mu = exc ? a.we_mu : a.wi_mu;
    const double sigma = exc ? a.we_sigma : a.wi_sigma;
    for (int r = 0; r < nn; ++r) {
      const int32_t tc = a.col_nbr[g * kMaxNbr + r];
      const uint64_t thr = a.col_thr[g * kMaxNbr + r];
      const uint32_t tl0 = (uint32_t)(a.col_local[tc] * a.npc);
      const uint32_t prank = (uint32_t)a.col_prank[g * kMaxNbr + r];
      // lane q holds the write cursor of segment (q, r)
      int32_t cursor = lane < a.nd ? L.seg[lane][r] : 0;
      for (int kb = 0; kb < a.npc; kb += 64) {
        const int k = kb + lane;
        int dd;
        Rand4 r4;
        const bool conn = decide(a, i, (int64_t)tc * a.npc + k, tl0 + (uint32_t)k, il, k0, k1,
                                 thr, k < a.npc, dd, r4);
        int32_t pos = 0;
        for (int q = 0; q < a.nd; ++q) {
          const unsigned long long m = __ballot(conn && dd == q);
          const int32_t cb = __shfl(cursor, q);
          if (conn && dd == q) pos = cb + __popcll(m & lt);
          if (lane == q) cursor += __popcll(m);
        }
        if (conn) {
          const Rand4 r2 = philox10(tl0 + (uint32_t)k, il, 1u, kStreamSyn, k0, k1);
          const uint32_t words[6] = {r4.z, r4.w, r2.x, r2.y, r2.z, r2.w};
          int32_t sum = 0;
#pragma unroll
          for (int q = 0; q < 6; ++q) sum += (int32_t)(words[q] & 0xffffu) + (int32_t)(words[q] >> 16);
          const double z = (double)(sum - 393210) * (1.0 / 65536.0);
          const double prod = sigma * z;
          const double w = mu + prod;
          const int16_t wq = (int16_t)__builtin_rint(w * 16384.0);
          out[pos] = (uint32_t)k | (prank << 12) | ((uint32_t)(uint16_t)wq << 16);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

GenArgs gen_args(const sim& s, int64_t row0, int64_t rows) {
  GenArgs a{};
  a.npc = s.npc;
  a.n_exc = s.cfg.n_exc;
  a.nd = s.nd;
  a.d_min = s.cfg.d_min;
  a.row0 = row0;
  a.rows = rows;
  a.col_net = s.col_net;
  a.col_local = s.col_local;
  a.col_nbr = s.col_nbr;
  a.col_nn = s.col_nn;
  a.col_part = s.col_part;
  a.col_prank = s.col_prank;
  a.col_np = s.col_np;
  a.col_pbase = s.col_pbase;
  a.col_thr = s.col_thr;
  a.net_key = s.net_key;
  a.we_mu = s.cfg.we_mu;
  a.we_sigma = s.cfg.we_sigma;
  a.wi_mu = s.cfg.wi_mu;
  a.wi_sigma = s.cfg.wi_sigma;
  a.row_base = s.row_base;
  a.syn = s.syn;
  a.idx = s.idx;
  a.idxw = s.idxw;
  a.deg = s.deg;
  return a;
}

int gen_grid(int64_t rows, int waves) {
  const int64_t wgs = (rows + waves - 1) / waves;
  return (int)(wgs < 65536 ? wgs : 65536);
}

// The 3x3 stencil's tables are small enough for four rows per workgroup; the 7x7 stencil's
// for two.
constexpr int kGenWaves3x3 = 4;
constexpr int kGenWavesWide = 2;

// ---- exclusive scan int32 -> int64 (three passes) ------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ int64_t block_exclusive_scan(int64_t x, int64_t* total) {
  __shared__ int64_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* in, int64_t n,
                                                              int64_t* part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t acc = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t e = base + (int64_t)q * kScanThreads + threadIdx.x;
    if (e < n) acc += in[e];
  }
  int64_t total;
  block_exclusive_scan(acc, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(int64_t* part, int64_t np) {
  int64_t carry = 0;
  for (int64_t b = 0; b < np; b += kScanThreads) {
    const int64_t e = b + threadIdx.x;
    const int64_t x = e < np ? part[e] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(x, &total);
    if (e < np) part[e] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* in, int64_t n,
                                                             const int64_t* part, int64_t* out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // each thread owns kScanItems consecutive elements
  const int64_t my0 = base + (int64_t)threadIdx.x * kScanItems;
  int64_t local = 0;
  for (int q = 0; q < kScanItems; ++q)
    if (my0 + q < n) local += in[my0 + q];
  int64_t total;
  int64_t run = part[blockIdx.x] + block_exclusive_scan(local, &total);
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t e = my0 + q;
    if (e < n) {
      out[e] = run;
      run += in[e];
      if (e == n - 1) out[n] = run;  // the total, written by the owner of the last element
    }
  }
}

}  // namespace

int64_t scan_scratch_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_gen_count(const sim& s, int64_t row0, int64_t rows, int32_t* row_len) {
  GenArgs a = gen_args(s, row0, rows);
  a.row_len = row_len;
  if (s.max_nn <= kMaxNbr3x3)
    hipLaunchKernelGGL((k_gen_count<kMaxNbr3x3, kGenWaves3x3>), dim3(gen_grid(rows, kGenWaves3x3)),
                       dim3(64 * kGenWaves3x3), 0, s.stream, a);
  else
    hipLaunchKernelGGL((k_gen_count<kMaxNbr, kGenWavesWide>), dim3(gen_grid(rows, kGenWavesWide)),
                       dim3(64 * kGenWavesWide), 0, s.stream, a);
  return hipGetLastError();
}

hipError_t launch_gen_fill(const sim& s, int64_t row0, int64_t rows) {
  GenArgs a = gen_args(s, row0, rows);
  if (s.max_nn <= kMaxNbr3x3)
    hipLaunchKernelGGL((k_gen_fill<kMaxNbr3x3, kGenWaves3x3>), dim3(gen_grid(rows, kGenWaves3x3)),
                       dim3(64 * kGenWaves3x3), 0, s.stream, a);
  else
    hipLaunchKernelGGL((k_gen_fill<kMaxNbr, kGenWavesWide>), dim3(gen_grid(rows, kGenWavesWide)),
                       dim3(64 * kGenWavesWide), 0, s.stream, a);
  return hipGetLastError();
}

// out[0..n] = exclusive prefix of in[0..n), out[n] = total.
// Row starts moved column by column: row i of column g starts at new_start[g] plus its
// offset inside the column (its scanned start minus the column's first).
__global__ __launch_bounds__(256) void k_fold_rows(int64_t* row_base, int64_t n, int32_t npc,
                                                   const int64_t* old_start,
                                                   const int64_t* new_start) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t g = i / npc;
    row_base[i] = new_start[g] + (row_base[i] - old_start[g]);
  }
}

hipError_t launch_fold_rows(const sim& s, const int64_t* old_start, const int64_t* new_start) {
  int64_t blocks = (s.n_neurons + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)blocks), dim3(256), 0, s.stream, s.row_base,
                     s.n_neurons, s.npc, old_start, new_start);
  return hipGetLastError();
}

hipError_t launch_scan_rows(const sim& s, const int32_t* in, int64_t n, int64_t* out,
                            int64_t* part, int64_t part_len) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb + 1 > part_len) return hipErrorInvalidValue;
  if (nb == 0) return hipMemsetAsync(out, 0, sizeof(int64_t), s.stream);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s.stream, in, n,
                     part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s.stream, part, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s.stream, in, n,
                     part, out);
  return hipGetLastError();
}

}  // namespace dpsnn
