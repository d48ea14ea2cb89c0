// noalloc.hip -- sim_read_spikes_static: sim_read_spikes without any allocation.
//
// sim_read_spikes of one network of a multi-network simulation finds the network's ranges in
// the recorded raster on the device and copies only those ids to the host; its scratch (the
// per-step ranges and the gathered ids) is allocated per call.  Callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid allocation) use
// this variant, whose scratch is the file-scope device array below: kStaticScratchBytes per
// device, held until the process ends.  Every call on one device shares that device's array,
// and each call overwrites what it uses of it (nothing needs to start at zero), so calls that
// overlap on one device race; the host side uses only the caller's buffers.
#include <mutex>
#include <string>

#include "dpsnn_internal.h"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Device address of `scratch` on each device, looked up once per device with that device
// current (in host code the array's name is only a stand-in for the symbol).
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" int sim_read_spikes_static(sim_t* s, int32_t net, int64_t t0, int64_t t1,
                                      int64_t* step_offsets, int32_t* ids, int64_t ids_cap,
                                      int64_t* n_ids) {
  if (!s) return DPSNN_EINVAL;
  auto fail = [&](int code, const char* msg) {
    s->err = msg;
    return code;
  };
  auto hip_fail = [&](const char* what, hipError_t e) {
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    return DPSNN_EHIP;
  };
  if (net < 0 || net >= s->n_nets) return fail(DPSNN_EINVAL, "net out of range");
  if (!s->ras_off) return fail(DPSNN_ESTATE, "spike recording is off");
  const int64_t lim = s->now < s->cfg.record_steps ? s->now : s->cfg.record_steps;
  if (t0 < 0 || t1 < t0 || t1 > lim) return fail(DPSNN_EINVAL, "steps outside the recorded window");
  if (!step_offsets || !n_ids) return fail(DPSNN_EINVAL, "NULL output");
  const int64_t ns = t1 - t0;
  const size_t step_bytes = align256(sizeof(int64_t) * 3 * (size_t)ns);
  if (step_bytes > kStaticScratchBytes)
    return fail(DPSNN_EINVAL, "step range exceeds the static scratch (16 MiB: 24 bytes per step)");
  const int rc = sim_sync(s);  // a sticky step failure leaves the recorded raster readable
  if (rc == DPSNN_ETRUNC || rc == DPSNN_EHIP) return rc;
  hipError_t e;
  if (s->n_nets == 1) {
    // one network holds every id: the recorded rows are the answer as they stand
    if ((e = hipMemcpy(step_offsets, s->ras_off + t0, sizeof(int64_t) * (size_t)(ns + 1),
                       hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail("raster offsets copy", e);
    const int64_t first = step_offsets[0];
    for (int64_t i = 0; i <= ns; ++i) step_offsets[i] -= first;
    const int64_t cnt = step_offsets[ns];
    *n_ids = cnt;
    const int64_t n = ids ? (cnt < ids_cap ? cnt : ids_cap) : 0;
    if (n > 0 && (e = hipMemcpy(ids, s->ras_ids + first, sizeof(int32_t) * (size_t)n,
                                hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail("raster ids copy", e);
    if (cnt > ids_cap || (!ids && cnt > 0)) return fail(DPSNN_ETRUNC, "ids buffer too small");
    return DPSNN_OK;
  }
  // several networks: per-step ranges [2 ns] and lengths / offsets [ns] in the first part of
  // the scratch, the gathered ids after it
  void* base = nullptr;
  if ((e = scratch_on(s->device, &base)) != hipSuccess) return hip_fail("hipGetSymbolAddress", e);
  int64_t* bounds = (int64_t*)base;
  int64_t* lens = bounds + 2 * ns;
  int32_t* take = (int32_t*)((unsigned char*)base + step_bytes);
  const int32_t lo = s->net_col0[net] * s->npc, hi = s->net_col0[net + 1] * s->npc;
  int64_t cnt = 0;
  if (ns > 0) {
    if ((e = dpsnn::launch_raster_bounds(*s, t0, ns, lo, hi, bounds)) != hipSuccess ||
        (e = dpsnn::launch_raster_lengths(*s, ns, bounds, lens)) != hipSuccess)
      return hip_fail("raster bounds", e);
    // the lengths land in the caller's offsets, which then become their exclusive prefix
    if ((e = hipMemcpyAsync(step_offsets, lens, sizeof(int64_t) * (size_t)ns,
                            hipMemcpyDeviceToHost, s->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(s->stream)) != hipSuccess)
      return hip_fail("raster lengths copy", e);
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t len = step_offsets[i];
      step_offsets[i] = cnt;
      cnt += len;
    }
  }
  step_offsets[ns] = cnt;
  *n_ids = cnt;
  const int64_t n = ids ? (cnt < ids_cap ? cnt : ids_cap) : 0;
  if (n > 0) {
    if (step_bytes + sizeof(int32_t) * (size_t)n > kStaticScratchBytes)
      return fail(DPSNN_EINVAL,
                  "ids exceed the static scratch (16 MiB: 24 bytes per step + 4 bytes per id)");
    if ((e = hipMemcpyAsync(lens, step_offsets, sizeof(int64_t) * (size_t)ns,
                            hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
        (e = dpsnn::launch_raster_take(*s, ns, bounds, lens, lo, n, take)) != hipSuccess ||
        (e = hipMemcpyAsync(ids, take, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                            s->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(s->stream)) != hipSuccess)
      return hip_fail("raster ids gather", e);
  }
  if (cnt > ids_cap || (!ids && cnt > 0)) return fail(DPSNN_ETRUNC, "ids buffer too small");
  return DPSNN_OK;
}
