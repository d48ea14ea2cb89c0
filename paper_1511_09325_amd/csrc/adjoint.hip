// adjoint.hip -- surrogate-gradient backpropagation through time of the step (train mode).
//
// Forward quantities of neuron j at step u (recorded by the forward or by the recompute of a
// checkpoint segment): V(u-1), Ca(u-1), the pre-threshold potential V~(u), the spike s(u) and the
// refractory flag r(u).  With nu(u) = dL/dV~(u), lambda(u) = dL/dV(u), mu(u) = dL/dCa(u):
//     e(u)  = dL/ds(u) + sum_{k in row(j)} w_k nu_{tgt k}(u + d_k)
//             + lambda(u) (V_reset - V~(u)) + alpha mu(u)
//     nu(u) = (1 - r(u)) [ lambda(u) (1 - s(u)) + e(u) sigma'(V~(u) - theta) ]
//     lambda(u-1) = P_m nu(u),   mu(u-1) = -gamma nu(u) + P_c mu(u)
//     dL/dw_k += nu_{tgt k}(u + d_k) at every spike of k's source,
//     dL/dP_m += V(u-1) nu(u),   dL/dgamma -= Ca(u-1) nu(u)
// with sigma'(x) = 1 / (1 + beta |x|)^2 (fast-sigmoid surrogate) and w_k the efficacy the
// forward delivered (the int32 rint(w 2^16) of the master weight, back in mV: straight-through
// rounding, so the recursion is the exact one of the forward that ran).  Per reverse step: the
// gather over every outgoing row from the ring of future nu (with the weight gradient of the
// rows whose neuron spiked) and k_adj_neuron (the recursion).  The gather is k_adj_col when
// every part of a row holds the synapses into one column (single-column native tiles: one
// workgroup per target column stages that column's future nu in LDS, one lane group per
// part; the synapses of delays of at least kAdjWindow are streamed once per window of
// kAdjWindow reverse steps, the shorter ones once per step), else k_adj_row (one wave per
// neuron, nu gathered from the ring).
// Everything is float32 except the per-neuron float64 partials of the two scalar
// gradients; every sum has a fixed order, so the result is deterministic.
#include <algorithm>

#include "dpsnn_internal.h"

namespace dpsnn {
namespace {

struct AdjArgs {
  StepArgs a;
  const int32_t* wfx;  // int32 efficacies of the forward, 2^-16 mV (rint of the master weight)
  float* gw;
  float* nu_ring;     // [dh][N]
  const uint8_t* dlyw; // [S'/4] delay index of each 16-byte word of records (groups are
                       // padded to whole words, so the four records of a word share it)
  float* gsum;        // [N]
  float* lam;         // [N]
  float* mu;          // [N]
  double* part;       // [2][N]: dL/dP_m, dL/dgamma partials
  const float* grad_rates;  // [n_cols]
  const int4* in_part;      // [C][9]: i-th source column of column C: (column, its global part
                            // into C, its first part, its part count)
  const int32_t* in_own;    // [C]: position of C itself among its source columns
  float* psum;              // [parts][npc]: sum over each part (k_adj_col), else null
  float* hsum;              // [kAdjWindow][parts][npc]: heavy-pass sums of a window
  int64_t n_idx;            // parts * npc
  float dlds_scale;   // dR_c / ds = 1000 / (npc T dt)
  float beta;
};

constexpr int kAdjUnroll = 8;  // records per lane in flight

// The weights the adjoint multiplies by are the ones the forward used: its int32 efficacies
// (rint of the master weight at 2^-16 mV) back in mV, exactly (|efficacy| < 2^24).  The
// gradient still goes to the float32 master weight unchanged (straight-through rounding).
__device__ __forceinline__ float4 efficacies_mv(int4 q) {
  return make_float4((float)q.x * 0x1p-16f, (float)q.y * 0x1p-16f, (float)q.z * 0x1p-16f,
                     (float)q.w * 0x1p-16f);
}

// One wave per neuron.  Each part of the row is streamed 64 x kAdjUnroll records at a time
// with each record's delay index from the train-mode delay array (one byte per 16-byte
// word), which selects the slot of the adjoint ring; the part's column table turns each
// record's rank into its target column.
__global__ __launch_bounds__(256) void k_adj_row(AdjArgs x, int64_t u) {
  const StepArgs& a = x.a;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int64_t j = (int64_t)blockIdx.x * 4 + wv;
  if (j >= nall) return;
  const int32_t g = (int32_t)(j / a.npc);
  const int32_t kk = (int32_t)(j - (int64_t)g * a.npc);
  const bool spiked = (a.rec_flags[(u - a.rec_base) * nall + j] & 1) != 0;
  const int32_t ubase = (int32_t)((u + a.d_min) % a.dh);  // ring slot of delay index 0
  float acc = 0.0f;
  for (int p = 0; p < a.col_np[g]; ++p) {
  const uint8_t* ent = idx_entry(a, g, kk, p);
  const int64_t rb = ent_start(ent);
  const int32_t rlen = ent_goff(ent)[a.nd];
  const int32_t* pcol = a.part_col + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
  for (int32_t f0 = 0; f0 < rlen; f0 += 64 * kAdjUnroll) {
    uint32_t w[kAdjUnroll];
    float wf[kAdjUnroll];
    int32_t dd[kAdjUnroll];
#pragma unroll
    for (int i = 0; i < kAdjUnroll; ++i) {
      const int32_t f = f0 + lane + 64 * i;
      w[i] = kDummyRecord;
      wf[i] = 0.0f;
      dd[i] = 0;
      if (f < rlen) {
        w[i] = a.syn[rb + f];
        wf[i] = (float)x.wfx[rb + f] * 0x1p-16f;
        dd[i] = x.dlyw[(rb + f) >> 2];
      }
    }
    float nu[kAdjUnroll];
#pragma unroll
    for (int i = 0; i < kAdjUnroll; ++i) {
      nu[i] = 0.0f;
      if (rec_rank(w[i]) != (uint32_t)kDummyRank) {
        const int32_t tc = pcol[rec_rank(w[i])];
        int32_t slot = ubase + dd[i];
        if (slot >= a.dh) slot -= a.dh;
        nu[i] = x.nu_ring[slot * nall + (int64_t)tc * a.npc + rec_k(w[i])];
      }
    }
#pragma unroll
    for (int i = 0; i < kAdjUnroll; ++i) {
      const int32_t f = f0 + lane + 64 * i;
      if (rec_rank(w[i]) == (uint32_t)kDummyRank) continue;
      const float prod = wf[i] * nu[i];
      acc = acc + prod;
      if (spiked) x.gw[rb + f] = x.gw[rb + f] + nu[i];
    }
  }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc = acc + __shfl_down(acc, off);
  if (lane == 0) x.gsum[j] = acc;
}

// Gather by target column (single-column parts).  Workgroup (x, tc) stages nu of column tc
// for a range of steps in LDS; then groups of LPP lanes take parts into tc (the synapses of
// one source neuron into tc) and stream them in 16-byte words (lane l of the group: words l,
// l + LPP, ...), summing w nu per lane in record order and then over the group by a fixed
// butterfly; where the source neuron spiked, nu is added to each synapse's gradient.  A
// column's own part holds most of a row (the in-column connection probability is the
// largest), so the first workgroups give a wave to each part of the own column and the rest a
// quad to each part of a neighbour.
//
// The reverse steps go in windows of up to kAdjWindow steps, top down to top - kw + 1.  A
// synapse of delay d >= kAdjWindow reaches, from every step t of the window, nu(t + d) with
// t + d > top: known when the window starts.  So the heavy pass streams the groups of those
// delays once per window with one sum per step of the window (nu of steps top + 1 + sb ..
// top + d_max staged), and a light pass per step streams only the groups of the shorter
// delays (nu of steps t + d_min .. t + kAdjWindow - 1, computed inside the window) and stores
// the part's sum as heavy + light.  Every step's sum is split the same way whatever window it
// falls in, and each synapse's gradient receives its terms one step after the other in
// decreasing step order, so the result does not depend on where windows or checkpoint
// segments begin.
constexpr int kAdjWords = 4;      // 16-byte words per lane in flight
constexpr int kAdjOwnPerWave = 16;   // own-column parts per wave
constexpr int kAdjNbrPerQuad = 4;    // neighbour parts per quad (one looked up per lane)

// One lane's share of a part's stream (see k_adj_col): adds the lane's w nu to acc[j] for
// every step j of the window (nu at staged index dd + ioff - j); spk bit j says the source
// neuron spiked at step top - j.
template <int LPP>
__device__ __forceinline__ void adj_stream(const AdjArgs& x, const float* nus, int npc,
                                           int64_t base, int32_t nwords, uint32_t spk, int gl,
                                           int kw, int32_t ioff, float (&acc)[kAdjWindow]) {
  for (int32_t w0 = gl; w0 < nwords; w0 += LPP * kAdjWords) {
    uint4 w[kAdjWords];
    float4 wf[kAdjWords];
    int32_t ddw[kAdjWords];
#pragma unroll
    for (int m = 0; m < kAdjWords; ++m) {
      const int32_t wi = w0 + LPP * m;
      const int64_t r = base + 4 * (int64_t)wi;
      w[m] = make_uint4(kDummyRecord, kDummyRecord, kDummyRecord, kDummyRecord);
      wf[m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      ddw[m] = kAdjWindow - 1 - ioff;  // an in-range index for absent words
      if (wi < nwords) {
        w[m] = *(const uint4*)(x.a.syn + r);
        wf[m] = efficacies_mv(*(const int4*)(x.wfx + r));
        ddw[m] = x.dlyw[r >> 2];
      }
    }
#pragma unroll
    for (int m = 0; m < kAdjWords; ++m) {
      const uint32_t rw[4] = {w[m].x, w[m].y, w[m].z, w[m].w};
      const float rf[4] = {wf[m].x, wf[m].y, wf[m].z, wf[m].w};
      const int32_t wi = w0 + LPP * m;
      const bool upd = spk != 0u && wi < nwords;
      float4* gp = (float4*)(x.gw + base + 4 * (int64_t)wi);
      float g[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (upd) {
        const float4 gv = *gp;
        g[0] = gv.x;
        g[1] = gv.y;
        g[2] = gv.z;
        g[3] = gv.w;
      }
#pragma unroll
      for (int j = 0; j < kAdjWindow; ++j) {
        if (j >= kw) break;
        const float* nj = nus + (ddw[m] + ioff - j) * npc;
        const bool sj = ((spk >> j) & 1u) != 0u;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (rec_rank(rw[c]) != (uint32_t)kDummyRank) {
            const float nu = nj[(int)rec_k(rw[c])];
            acc[j] = acc[j] + rf[c] * nu;
            if (sj) g[c] = g[c] + nu;
          }
        }
      }
      if (upd) *gp = make_float4(g[0], g[1], g[2], g[3]);
    }
  }
}

// A lane's part, looked up ahead: first word of its groups g_lo .. g_hi - 1, their length in
// 16-byte words, the source neuron's spikes at steps u, u - 1, .. u - kw + 1 (bit j), and
// where the part's sum goes.
struct AdjPart {
  int64_t base;
  int32_t nwords;
  uint32_t spk;
  int64_t out;
};

__device__ __forceinline__ AdjPart adj_lookup(const AdjArgs& x, int64_t u, int4 in, int32_t kk,
                                              int g_lo, int g_hi, int kw) {
  const StepArgs& a = x.a;
  const int npc = a.npc;
  const int64_t nall = (int64_t)a.n_cols * npc;
  const int32_t src = in.x, q = in.y, pf = in.z, np = in.w;
  const uint8_t* ent = a.idx + ((int64_t)npc * pf + (int64_t)kk * np + (q - pf)) * a.idxw;
  AdjPart P;
  P.base = ent_start(ent) + ent_goff(ent)[g_lo];
  P.nwords = (ent_goff(ent)[g_hi] - ent_goff(ent)[g_lo]) >> 2;
  P.spk = 0u;
  for (int j = 0; j < kw; ++j)
    P.spk |= (uint32_t)(a.rec_flags[(u - j - a.rec_base) * nall + (int64_t)src * npc + kk] & 1) << j;
  P.out = (int64_t)q * npc + kk;
  return P;
}

// Group of LPP lanes taking PPG parts, one after the other: lane gl < PPG looks up part gl
// first (all the lookups in one round of loads), then the group streams part r with lane r's
// lookup, sums over the group by a fixed butterfly and stores the part's sums, one per step
// of the window, into hsum.
template <int LPP, int PPG>
__device__ __forceinline__ void adj_group(const AdjArgs& x, const float* nus, const AdjPart& mine,
                                          bool mine_ok, int kw, int32_t ioff) {
  static_assert(PPG <= LPP, "each lane of a group looks up one of its parts");
  const int lane = threadIdx.x & 63, gl = lane & (LPP - 1), g0 = lane - gl;
  const int npc = x.a.npc;
  for (int r = 0; r < PPG; ++r) {
    const int okr = __shfl((int32_t)mine_ok, g0 + r);
    if (!okr) break;  // uniform over the group; parts are assigned in order
    const int64_t base = ((int64_t)__shfl((int32_t)(mine.base >> 32), g0 + r) << 32) |
                         (uint32_t)__shfl((int32_t)(uint32_t)mine.base, g0 + r);
    const int32_t nwords = __shfl(mine.nwords, g0 + r);
    const uint32_t spk = (uint32_t)__shfl((int32_t)mine.spk, g0 + r);
    float acc[kAdjWindow];
#pragma unroll
    for (int j = 0; j < kAdjWindow; ++j) acc[j] = 0.0f;
    adj_stream<LPP>(x, nus, npc, base, nwords, spk, gl, kw, ioff, acc);
#pragma unroll
    for (int j = 0; j < kAdjWindow; ++j)
#pragma unroll
      for (int off = LPP / 2; off > 0; off >>= 1) acc[j] = acc[j] + __shfl_xor(acc[j], off, LPP);
    const int64_t out = ((int64_t)__shfl((int32_t)(mine.out >> 32), g0 + r) << 32) |
                        (uint32_t)__shfl((int32_t)(uint32_t)mine.out, g0 + r);
    if (gl == 0) {
#pragma unroll
      for (int j = 0; j < kAdjWindow; ++j)
        if (j < kw) x.hsum[(int64_t)j * x.n_idx + out] = acc[j];
    }
  }
}

// Heavy pass, workgroup (x, tc): stages nu of column tc for nst steps from step st0, then
// streams its share of the parts into tc, groups g_lo .. g_hi - 1 of each, for the steps u ..
// u - kw + 1 of a window.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_adj_col(AdjArgs x, int64_t u, int32_t nbw, int32_t g_lo,
                                                   int32_t g_hi, int32_t kw, int32_t nst,
                                                   int64_t st0, int32_t ioff) {
  extern __shared__ float nus[];  // [nst][npc]
  const StepArgs& a = x.a;
  constexpr int NW = BLOCK / 64, NQ = BLOCK / 4;
  const int32_t tc = blockIdx.y;
  const int npc = a.npc;
  const int nn = a.col_nn[tc];
  const bool own = (int32_t)blockIdx.x < nbw;
  const int32_t first = own ? (int32_t)blockIdx.x * NW * kAdjOwnPerWave
                            : ((int32_t)blockIdx.x - nbw) * NQ * kAdjNbrPerQuad;
  const int32_t nparts = own ? npc : (nn - 1) * npc;
  if (first >= nparts) return;
  const int i_own = x.in_own[tc];
  // this lane's part, looked up before the staging so that the loads overlap
  const int lane = threadIdx.x & 63;
  AdjPart mine{0, 0, 0u, 0};
  bool mine_ok = false;
  if (own) {
    const int gl = lane;
    const int32_t kk = first + (threadIdx.x >> 6) * kAdjOwnPerWave + gl;
    if (gl < kAdjOwnPerWave && kk < npc) {
      mine = adj_lookup(x, u, x.in_part[tc * kMaxNbr + i_own], kk, g_lo, g_hi, kw);
      mine_ok = true;
    }
  } else {
    const int gl = lane & 3;
    const int32_t e = first + gl * NQ + (threadIdx.x >> 2);
    if (e < nparts) {
      int i = e / npc;
      const int32_t kk = e - i * npc;
      if (i >= i_own) ++i;  // skip the own column
      mine = adj_lookup(x, u, x.in_part[tc * kMaxNbr + i], kk, g_lo, g_hi, kw);
      mine_ok = true;
    }
  }
  // staging, kStage loads in flight per thread; e / npc through a float reciprocal (exact:
  // e < 2^16)
  const int64_t nall = (int64_t)a.n_cols * npc;
  const int32_t slot0 = (int32_t)(st0 % a.dh);
  const float inv_npc = 1.0f / (float)npc;
  const int32_t ntot = nst * npc;
  constexpr int kStage = 8;
  for (int32_t e0 = threadIdx.x; e0 < ntot; e0 += BLOCK * kStage) {
    float v[kStage];
#pragma unroll
    for (int m = 0; m < kStage; ++m) {
      const int32_t e = e0 + m * BLOCK;
      v[m] = 0.0f;
      if (e < ntot) {
        const int dd = (int)(((float)e + 0.5f) * inv_npc), k = e - dd * npc;
        int32_t slot = slot0 + dd;
        if (slot >= a.dh) slot -= a.dh;
        v[m] = x.nu_ring[(int64_t)slot * nall + (int64_t)tc * npc + k];
      }
    }
#pragma unroll
    for (int m = 0; m < kStage; ++m)
      if (e0 + m * BLOCK < ntot) nus[e0 + m * BLOCK] = v[m];
  }
  __syncthreads();
  if (own) adj_group<64, kAdjOwnPerWave>(x, nus, mine, mine_ok, kw, ioff);
  else adj_group<4, kAdjNbrPerQuad>(x, nus, mine, mine_ok, kw, ioff);
}

// Light pass of step t, the jl-th of its window: a quad per part into column tc (blockIdx.y)
// streams the part's groups 0 .. hsplit - 1 (the delays shorter than the window) with nu read
// from the ring (the steps t + d_min .. t + kAdjWindow - 1, computed inside the window), adds
// nu to the gradient where the source neuron spiked at t, and stores heavy + light as the
// part's sum.  The quad's sum is its lanes' sums in word order by a fixed butterfly.
__global__ __launch_bounds__(256) void k_adj_light(AdjArgs x, int64_t t, int32_t hsplit,
                                                   int32_t jl) {
  const StepArgs& a = x.a;
  const int npc = a.npc;
  const int32_t tc = blockIdx.y;
  const int32_t e = (int32_t)blockIdx.x * 64 + (int32_t)(threadIdx.x >> 2);
  const int gl = threadIdx.x & 3;
  if (e >= a.col_nn[tc] * npc) return;  // whole quads
  const int i = e / npc;
  const int32_t kk = e - i * npc;
  const int4 in = x.in_part[tc * kMaxNbr + i];
  const int64_t nall = (int64_t)a.n_cols * npc;
  const uint8_t* ent = a.idx + ((int64_t)npc * in.z + (int64_t)kk * in.w + (in.y - in.z)) * a.idxw;
  const int64_t base = ent_start(ent) + ent_goff(ent)[0];
  const int32_t nwords = (ent_goff(ent)[hsplit] - ent_goff(ent)[0]) >> 2;
  const bool spiked = (a.rec_flags[(t - a.rec_base) * nall + (int64_t)in.x * npc + kk] & 1) != 0;
  const int64_t out = (int64_t)in.y * npc + kk;
  const float h = x.hsum[(int64_t)jl * x.n_idx + out];
  const int32_t slot0 = (int32_t)((t + a.d_min) % a.dh);
  const float* col_nu = x.nu_ring + (int64_t)tc * npc;
  float acc = 0.0f;
  for (int32_t w0 = gl; w0 < nwords; w0 += 4 * kAdjWords) {
    uint4 w[kAdjWords];
    float4 wf[kAdjWords];
    int32_t ddw[kAdjWords];
#pragma unroll
    for (int m = 0; m < kAdjWords; ++m) {
      const int32_t wi = w0 + 4 * m;
      const int64_t r = base + 4 * (int64_t)wi;
      w[m] = make_uint4(kDummyRecord, kDummyRecord, kDummyRecord, kDummyRecord);
      wf[m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      ddw[m] = 0;
      if (wi < nwords) {
        w[m] = *(const uint4*)(a.syn + r);
        wf[m] = efficacies_mv(*(const int4*)(x.wfx + r));
        ddw[m] = x.dlyw[r >> 2];
      }
    }
#pragma unroll
    for (int m = 0; m < kAdjWords; ++m) {
      const uint32_t rw[4] = {w[m].x, w[m].y, w[m].z, w[m].w};
      const float rf[4] = {wf[m].x, wf[m].y, wf[m].z, wf[m].w};
      int32_t slot = slot0 + ddw[m];
      if (slot >= a.dh) slot -= a.dh;
      const float* nu_s = col_nu + (int64_t)slot * nall;
      float nu[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        nu[c] = 0.0f;
        if (rec_rank(rw[c]) != (uint32_t)kDummyRank) {
          nu[c] = nu_s[(int)rec_k(rw[c])];
          acc = acc + rf[c] * nu[c];
        }
      }
      const int32_t wi = w0 + 4 * m;
      if (spiked && wi < nwords) {
        float4* gp = (float4*)(x.gw + base + 4 * (int64_t)wi);
        float4 gv = *gp;
        if (rec_rank(rw[0]) != (uint32_t)kDummyRank) gv.x = gv.x + nu[0];
        if (rec_rank(rw[1]) != (uint32_t)kDummyRank) gv.y = gv.y + nu[1];
        if (rec_rank(rw[2]) != (uint32_t)kDummyRank) gv.z = gv.z + nu[2];
        if (rec_rank(rw[3]) != (uint32_t)kDummyRank) gv.w = gv.w + nu[3];
        *gp = gv;
      }
    }
  }
  acc = acc + __shfl_xor(acc, 2, 4);
  acc = acc + __shfl_xor(acc, 1, 4);
  if (gl == 0) x.psum[out] = h + acc;
}

// Delay index of every 16-byte word of records (train mode): one wave per neuron over its
// parts and groups (parts and groups start on whole words).
__global__ __launch_bounds__(256) void k_fill_dly(StepArgs a, uint8_t* dlyw) {
  const int lane = threadIdx.x & 63;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < nall;
       i += (int64_t)gridDim.x * 4) {
    const int32_t g = (int32_t)(i / a.npc);
    const int32_t kk = (int32_t)(i - (int64_t)g * a.npc);
    for (int p = 0; p < a.col_np[g]; ++p) {
      const uint8_t* ent = idx_entry(a, g, kk, p);
      const int64_t st = ent_start(ent);
      const uint16_t* go = ent_goff(ent);
      for (int d = 0; d < a.nd; ++d)
        for (int32_t f = go[d] + 4 * lane; f < go[d + 1]; f += 4 * 64)
          dlyw[(st + f) >> 2] = (uint8_t)d;
    }
  }
}

__global__ __launch_bounds__(256) void k_adj_neuron(AdjArgs x, int64_t u) {
  const StepArgs& a = x.a;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  const int64_t uslot = u % a.dh;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < nall;
       j += (int64_t)gridDim.x * 256) {
    const int64_t o = (u - a.rec_base) * nall + j;
    const uint8_t fl = a.rec_flags[o];
    const float s = (fl & 1) ? 1.0f : 0.0f;
    const float vt = a.rec_vt[o];
    const float lam = x.lam[j], mu = x.mu[j];
    const int32_t g = (int32_t)(j / a.npc);
    const float dlds = x.grad_rates[g] * x.dlds_scale;
    float gsum;
    if (x.psum) {  // the parts' sums, in part order
      const int32_t kk = (int32_t)(j - (int64_t)g * a.npc), pf = a.col_pfirst[g];
      gsum = 0.0f;
      for (int p = 0; p < a.col_np[g]; ++p) gsum = gsum + x.psum[(int64_t)(pf + p) * a.npc + kk];
    } else {
      gsum = x.gsum[j];
    }
    const float reset_term = lam * (a.k.vreset - vt);
    const float e = ((dlds + gsum) + reset_term) + a.k.alpha * mu;
    float nu = 0.0f;
    if (!(fl & 2)) {
      const float den = 1.0f + x.beta * fabsf(vt - a.k.theta);
      const float sig = 1.0f / (den * den);
      nu = lam * (1.0f - s) + e * sig;
    }
    x.nu_ring[uslot * nall + j] = nu;
    x.part[j] += (double)a.rec_vprev[o] * (double)nu;
    x.part[nall + j] -= (double)a.rec_caprev[o] * (double)nu;
    x.lam[j] = a.k.pm * nu;
    x.mu[j] = a.k.pc * mu - a.k.gam * nu;
  }
}

// Sums of the two partial arrays in a fixed order (one workgroup).
__global__ __launch_bounds__(1024) void k_reduce_parts(const double* part, int64_t n,
                                                       double* out) {
  __shared__ double buf[2][1024];
  for (int c = 0; c < 2; ++c) {
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 1024) acc += part[c * n + e];
    buf[c][threadIdx.x] = acc;
  }
  __syncthreads();
  for (int width = 512; width > 0; width >>= 1) {
    if ((int)threadIdx.x < width) {
      buf[0][threadIdx.x] += buf[0][threadIdx.x + width];
      buf[1][threadIdx.x] += buf[1][threadIdx.x + width];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = buf[0][0];
    out[1] = buf[1][0];
  }
}

// Canonical synapse order (per source neuron: the real records sorted by (delay, target))
// <-> the padded device layout.  mode 0: dst_padded[p] = src_canon[c]; mode 1: the reverse;
// mode 2: rel[p] = c - canon_start[row] (the permutation that k_canon_apply replays).
// Padding records receive 0 in mode 0.  One wave per neuron (one per workgroup: the counts
// of the 7x7 stencil fill the LDS): the counts of its synapses per (delay, stencil rank)
// give the canonical start of every (delay, rank) run; inside a device group (part, delay)
// the runs of the part's ranks follow each other in rank order (part ranks are ascending
// stencil ranks, see part_srank).
__global__ __launch_bounds__(64) void k_canon_map(StepArgs a, const int64_t* canon_start,
                                                  int mode, const float* src, float* dst,
                                                  uint16_t* rel) {
  __shared__ int32_t cnt[kMaxDelay * kMaxNbr];
  __shared__ int64_t cst[kMaxDelay * kMaxNbr];
  const int lane = threadIdx.x & 63;
  const int64_t nall = (int64_t)a.n_cols * a.npc;
  for (int64_t i = blockIdx.x; i < nall; i += gridDim.x) {
    const int32_t g = (int32_t)(i / a.npc);
    const int32_t kk = (int32_t)(i - (int64_t)g * a.npc);
    const int np = a.col_np[g], nn = a.col_nn[g];
    for (int q = lane; q < kMaxDelay * kMaxNbr; q += 64) cnt[q] = 0;
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      const uint8_t* ent = idx_entry(a, g, kk, p);
      const int64_t st = ent_start(ent);
      const uint16_t* go = ent_goff(ent);
      const int32_t* srank = a.part_srank + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
      for (int dd = 0; dd < a.nd; ++dd)
        for (int32_t f = go[dd] + lane; f < go[dd + 1]; f += 64) {
          const uint32_t q = rec_rank(a.syn[st + f]);
          if (q != (uint32_t)kDummyRank) atomicAdd(&cnt[dd * kMaxNbr + srank[q]], 1);
        }
    }
    __syncthreads();
    if (lane == 0) {
      int64_t c = canon_start[i];
      for (int dd = 0; dd < a.nd; ++dd)
        for (int r = 0; r < nn; ++r) {
          cst[dd * kMaxNbr + r] = c;
          c += cnt[dd * kMaxNbr + r];
        }
    }
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      const uint8_t* ent = idx_entry(a, g, kk, p);
      const int64_t st = ent_start(ent);
      const uint16_t* go = ent_goff(ent);
      const int32_t* srank = a.part_srank + (int64_t)(a.col_pfirst[g] + p) * kMaxPartCols;
      for (int dd = 0; dd < a.nd; ++dd)
        for (int32_t f = go[dd] + lane; f < go[dd + 1]; f += 64) {
          const uint32_t q = rec_rank(a.syn[st + f]);
          if (q == (uint32_t)kDummyRank) {
            if (mode == 0) dst[st + f] = 0.0f;
            continue;
          }
          int32_t run0 = go[dd];
          for (int q2 = 0; q2 < (int)q; ++q2) run0 += cnt[dd * kMaxNbr + srank[q2]];
          const int64_t c = cst[dd * kMaxNbr + srank[q]] + (f - run0);
          if (mode == 0) dst[st + f] = src[c];
          else if (mode == 1) dst[c] = src[st + f];
          else rel[st + f] = (uint16_t)(c - canon_start[i]);
        }
    }
    __syncthreads();
  }
}

// The same maps from the stored permutation: one wave per row, its padded records in order
// (the parts of a row are contiguous, and the rows of one column follow each other; the last
// row of a column ends at the column's end); rel 0xffff marks padding (rows are shorter than
// 0xffff synapses: checked when train mode is set up).
__global__ __launch_bounds__(256) void k_canon_apply(const int64_t* row_base,
                                                     const int64_t* col_end, int32_t npc,
                                                     const int64_t* canon_start,
                                                     const uint16_t* rel, int64_t n_rows,
                                                     int mode, const float* src, float* dst) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n_rows;
       i += (int64_t)gridDim.x * 4) {
    const int64_t r0 = row_base[i], c0 = canon_start[i];
    const int64_t r1 = (i + 1) % npc == 0 ? col_end[i / npc] : row_base[i + 1];
    for (int64_t q = r0 + lane; q < r1; q += 64) {
      const uint32_t o = rel[q];
      if (o == 0xffffu) {
        if (mode == 0) dst[q] = 0.0f;
        continue;
      }
      if (mode == 0) dst[q] = src[c0 + o];
      else dst[c0 + o] = src[q];
    }
  }
}

// Initial master weights from the int16 records: w = w_q * 2^-14 mV (dummies 0).
__global__ void k_weights_from_records(const uint32_t* syn, float* w, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t r = syn[e];
    w[e] = rec_rank(r) == (uint32_t)kDummyRank ? 0.0f
                                               : (float)(int16_t)(r >> 16) * 0x1p-14f;
  }
}

__global__ void k_column_rates(const unsigned long long* col_spk, int32_t n_cols, float scale,
                               float* rates) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n_cols) rates[c] = (float)((double)col_spk[c] * (double)scale);
}

// The built-in loss of sim_backward: L = mean over columns of (R_c - R*_c)^2 and its
// gradient dL/dR_c = 2 (R_c - R*_c) / C.  One workgroup; the loss is summed in double in a
// fixed order (lane-strided partial sums, then a fixed tree), so it is deterministic.
__global__ __launch_bounds__(256) void k_rate_loss(const float* rates, const float* targets,
                                                   int32_t n_cols, float* loss, float* grad) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int32_t c = threadIdx.x; c < n_cols; c += 256) {
    const double d = (double)rates[c] - (double)targets[c];
    acc += d * d;
    grad[c] = (float)(2.0 * d / (double)n_cols);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = (float)(part[0] / (double)n_cols);
}

int grid_of(int64_t items, int per_block) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

namespace {

// Split of the delays between the heavy pass and the light passes of a window: groups
// dd < hsplit (delays below kAdjWindow) are light; the heavy pass stages nu of steps
// top + 1 + sb .. top + d_max.
struct AdjSplit {
  int32_t hsplit, sb, nst;
};

AdjSplit adj_split(int32_t nd, int32_t d_min, int32_t d_max) {
  AdjSplit p;
  p.hsplit = std::min(nd, std::max(0, kAdjWindow - d_min));
  p.sb = std::max(d_min, kAdjWindow) - kAdjWindow;
  p.nst = d_max - p.sb;
  return p;
}

AdjArgs adj_args(const sim& s, const float* grad_rates, float scale, float beta) {
  AdjArgs x{};
  x.a = make_step_args(s);
  // the trajectory of the segment being reversed
  x.a.rec_vprev = s.rec_vprev;
  x.a.rec_caprev = s.rec_caprev;
  x.a.rec_vt = s.rec_vt;
  x.a.rec_flags = s.rec_flags;
  x.a.rec_base = s.rec_base;
  x.wfx = s.wfx;
  x.gw = s.gw;
  x.nu_ring = s.nu_ring;
  x.dlyw = s.dlyw;
  x.gsum = s.adj_gsum;
  x.lam = s.adj_lam;
  x.mu = s.adj_mu;
  x.part = s.adj_part;
  x.grad_rates = grad_rates;
  x.dlds_scale = scale;
  x.beta = beta;
  if (s.adj_psum) {
    x.in_part = (const int4*)s.in_part;
    x.in_own = s.in_own;
    x.psum = s.adj_psum;
    x.hsum = s.adj_hsum;
    x.n_idx = s.n_idx;
  }
  return x;
}

}  // namespace

// Does the column-wise gather's heavy staging (nu of one column over up to d_max steps) fit
// the LDS?
bool adjoint_col_fits(int32_t npc, int32_t d_min, int32_t d_max) {
  const AdjSplit p = adj_split(d_max - d_min + 1, d_min, d_max);
  return sizeof(float) * (size_t)p.nst * (size_t)npc + 1024 <= kMaxLds;
}

// Reverse steps top, top - 1, .. down to at most lo (a window of up to kAdjWindow steps with
// the column-wise gather, one step otherwise); *next is the next step to reverse.  The steps
// must lie in the recorded segment.
hipError_t launch_adjoint_window(const sim& s, int64_t top, int64_t lo, const float* grad_rates,
                                 float scale, float beta, int64_t* next) {
  const AdjArgs x = adj_args(s, grad_rates, scale, beta);
  const dim3 gn(grid_of(s.n_neurons, 256));
  if (!s.adj_psum) {
    hipLaunchKernelGGL(k_adj_row, dim3((unsigned)((s.n_neurons + 3) / 4)), dim3(256), 0, s.stream,
                       x, top);
    hipLaunchKernelGGL(k_adj_neuron, gn, dim3(256), 0, s.stream, x, top);
    *next = top - 1;
    return hipGetLastError();
  }
  const int32_t kw = (int32_t)std::min<int64_t>(kAdjWindow, top - lo + 1);
  const int32_t d_min = s.cfg.d_min, d_max = s.cfg.d_max;
  const AdjSplit p = adj_split(s.nd, d_min, d_max);
  const int nbw = (s.npc + 16 * kAdjOwnPerWave - 1) / (16 * kAdjOwnPerWave);
  const int nbq = ((s.max_nn - 1) * s.npc + 256 * kAdjNbrPerQuad - 1) / (256 * kAdjNbrPerQuad);
  const dim3 gc((unsigned)(nbw + nbq), (unsigned)s.n_cols);
  // heavy pass: groups hsplit .. nd - 1 for the kw steps, staged index dd + d_min - 1 - sb - j
  hipLaunchKernelGGL(k_adj_col<1024>, gc, dim3(1024), sizeof(float) * (size_t)p.nst * s.npc,
                     s.stream, x, top, nbw, p.hsplit, s.nd, kw, p.nst, top + 1 + p.sb,
                     d_min - 1 - p.sb);
  // light passes: groups 0 .. hsplit - 1, a quad per part, 64 parts per workgroup
  const dim3 gl((unsigned)((s.max_nn * s.npc + 63) / 64), (unsigned)s.n_cols);
  for (int32_t j = 0; j < kw; ++j) {
    const int64_t t = top - j;
    hipLaunchKernelGGL(k_adj_light, gl, dim3(256), 0, s.stream, x, t, p.hsplit, j);
    hipLaunchKernelGGL(k_adj_neuron, gn, dim3(256), 0, s.stream, x, t);
  }
  *next = top - kw;
  return hipGetLastError();
}

// Allow the column-wise reverse gather the dynamic LDS beyond 64 KB (its nu staging).
hipError_t prepare_adjoint_kernels() {
  return hipFuncSetAttribute((const void*)k_adj_col<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kMaxLds);
}

hipError_t launch_reduce_parts(const sim& s, double* out) {
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(1024), 0, s.stream, s.adj_part, s.n_neurons,
                     out);
  return hipGetLastError();
}

hipError_t launch_canon_map(const sim& s, int mode, const float* src, float* dst) {
  if (s.canon_rel) {
    hipLaunchKernelGGL(k_canon_apply, dim3(grid_of(s.n_neurons, 4)), dim3(256), 0, s.stream,
                       s.row_base, s.col_end, s.npc, s.canon_start, s.canon_rel, s.n_neurons,
                       mode, src, dst);
    return hipGetLastError();
  }
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_canon_map, dim3(grid_of(s.n_neurons, 1)), dim3(64), 0, s.stream, a,
                     s.canon_start, mode, src, dst, nullptr);
  return hipGetLastError();
}

hipError_t launch_canon_perm(const sim& s, uint16_t* rel) {
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_canon_map, dim3(grid_of(s.n_neurons, 1)), dim3(64), 0, s.stream, a,
                     s.canon_start, 2, nullptr, nullptr, rel);
  return hipGetLastError();
}

hipError_t launch_fill_dly(const sim& s) {
  const StepArgs a = make_step_args(s);
  hipLaunchKernelGGL(k_fill_dly, dim3(grid_of(s.n_neurons, 4)), dim3(256), 0, s.stream, a, s.dlyw);
  return hipGetLastError();
}

hipError_t launch_weights_from_records(const sim& s) {
  hipLaunchKernelGGL(k_weights_from_records, dim3(grid_of(s.n_syn_padded, 256)), dim3(256), 0,
                     s.stream, s.syn, s.wf32, s.n_syn_padded);
  return hipGetLastError();
}

hipError_t launch_rate_loss(const sim& s, const float* rates, const float* targets, float* loss,
                            float* grad_rates) {
  hipLaunchKernelGGL(k_rate_loss, dim3(1), dim3(256), 0, s.stream, rates, targets, s.n_cols,
                     loss, grad_rates);
  return hipGetLastError();
}

hipError_t launch_column_rates(const sim& s, float scale, float* rates) {
  hipLaunchKernelGGL(k_column_rates, dim3(grid_of(s.n_cols, 256)), dim3(256), 0, s.stream,
                     s.col_spk, s.n_cols, scale, rates);
  return hipGetLastError();
}

}  // namespace dpsnn
