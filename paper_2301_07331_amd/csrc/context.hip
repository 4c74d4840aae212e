// context.hip -- the per-device context of libhlc: device state, the shared
// workspace, counters read-back, per-thread call statistics, and the
// entry points that are not a cross-match (error strings, statistics,
// shutdown).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "host.hpp"

namespace hlc {

Device g_dev[MAX_DEVICES];
thread_local hlc_stats g_stats;

int get_device(Device** out, int* dev_id) {
  int dev = 0;
  HLC_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return HLC_E_DEVICE;
  Device& d = g_dev[dev];
  if (!d.init) {
    HLC_TRY(hipMalloc(&d.cnt, sizeof(Counters)));
    HLC_TRY(hipHostMalloc(&d.cnt_host, sizeof(Counters), hipHostMallocDefault));
    for (auto& e : d.ev) HLC_TRY(hipEventCreate(&e));
    HLC_TRY(hipDeviceGetAttribute(&d.ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HLC_TRY(hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking));
    HLC_TRY(hipEventCreateWithFlags(&d.fork, hipEventDisableTiming));
    HLC_TRY(hipEventCreateWithFlags(&d.bsorted, hipEventDisableTiming));
    HLC_TRY(hipEventCreateWithFlags(&d.prepped, hipEventDisableTiming));
    HLC_TRY(hipHostMalloc(&d.fmsg_host, 64, hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(d.fmsg_host, 0, 64);
    HLC_TRY(hipHostGetDevicePointer((void**)&d.fmsg_dev, d.fmsg_host, 0));
    d.init = true;
  }
  *out = &d;
  if (dev_id) *dev_id = dev;
  return HLC_OK;
}

bool alloc_fails(size_t bytes) {
  if (const char* f = std::getenv("HLC_TEST_FAIL_ALLOC")) {
    long long lim = std::atoll(f);
    if (lim > 0 && bytes >= (size_t)lim) return true;
  }
  return false;
}

int dev_alloc(void** p, size_t bytes) {
  if (alloc_fails(bytes)) return HLC_E_NOMEM;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return HLC_E_NOMEM;
  }
  return HLC_OK;
}


int ensure_ws(Device& d, size_t bytes) {
  if (bytes <= d.ws_bytes) return HLC_OK;
  if (d.ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(d.ws);
    d.ws = nullptr;
    d.ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4 + (1 << 20);
  HLC_CHECK(dev_alloc(&d.ws, want));
  d.ws_bytes = want;
  return HLC_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

void fill_stats(const Counters& h, int64_t na, int64_t nb, int64_t nbh, const Geom& g) {
  std::memset(&g_stats, 0, sizeof(g_stats));
  g_stats.na = na;
  g_stats.nb = nb;
  g_stats.nb_halo = nbh;
  g_stats.n_pairs = (int64_t)h.n_pairs;
  g_stats.n_candidates = (int64_t)h.n_cand;
  g_stats.n_band = (int64_t)h.n_band;
  g_stats.n_ties = (int64_t)h.n_ties;
  g_stats.n_zones = g.nz;
  g_stats.ra_bits = g.rb;
  g_stats.zone_height_arcsec = g.h_deg * 3600.0;
}

// Stage times from the event slots: 0 start; 14 counters cleared; 5 A's
// keygen done (side stream) and 1 B's keygen done (call's stream, the two
// side by side); B's sort and
// layout 2-4 on the call's stream; A's sort 6 (and 7) on the side stream;
// 12 both sorts done, 8 ranges done (side stream, beside B's layout); 13
// filter start; 9 filter; 10 certification and packing; 11 end. Stages on
// the two streams overlap, so their times add up to more than the wall time.
void fill_times(Device& dev, bool with_partition) {
  auto el = [&](int a, int b) { return (double)elapsed(dev.ev[a], dev.ev[b]); };
  if (with_partition) {
    g_stats.t_keygen_ms = std::max(el(14, 5), el(14, 1));
    g_stats.t_sort_ms = el(2, 3) + el(5, 6);
    g_stats.t_layout_ms = el(3, 4) + el(6, 7);
    g_stats.t_ranges_ms = el(12, 8);
  } else {
    g_stats.t_ranges_ms = el(0, 8);
  }
  g_stats.t_match_ms = el(13, 9);
  g_stats.t_certify_ms = el(9, 10);
  g_stats.t_total_ms = el(0, 11);
}

int read_counters(Device& dev, hipStream_t s, bool prof) {
  HLC_TRY(hipMemcpyAsync(dev.cnt_host, dev.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
  if (prof) HLC_TRY(hipEventRecord(dev.ev[11], s));
  HLC_TRY(hipStreamSynchronize(s));
  HLC_TRY(hipGetLastError());
  return HLC_OK;
}

}  // namespace hlc

using namespace hlc;

extern "C" {

const char* hlc_strerror(int status) {
  switch (status) {
    case HLC_OK: return "ok";
    case HLC_E_INVAL: return "invalid argument or coordinate";
    case HLC_E_NOMEM: return "out of memory";
    case HLC_E_OVERFLOW: return "output capacity too small (required count returned)";
    case HLC_E_DEVICE: return "HIP runtime error";
    case HLC_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

int hlc_last_stats(hlc_stats* out) {
  if (!out) return HLC_E_INVAL;
  *out = g_stats;
  return HLC_OK;
}

void hlc_shutdown(void) {
  batch_release_all();
  for (auto& d : g_dev) {
    if (!d.init) continue;
    if (d.ws) (void)hipFree(d.ws);
    if (d.cnt) (void)hipFree(d.cnt);
    if (d.cnt_host) (void)hipHostFree(d.cnt_host);
    if (d.fmsg_host) (void)hipHostFree(d.fmsg_host);
    for (auto& e : d.ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {d.fork, d.bsorted, d.prepped})
      if (e) (void)hipEventDestroy(e);
    if (d.side) (void)hipStreamDestroy(d.side);
    for (void* p : d.sarena)
      if (p) (void)hipFree(p);
    if (d.harena) (void)hipHostFree(d.harena);
    d = Device();
  }
}

}  // extern "C"
