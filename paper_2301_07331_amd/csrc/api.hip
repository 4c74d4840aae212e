// api.hip -- the C ABI of libhlc: argument checks, partition geometry,
// per-device workspace, and the order of kernel launches for one call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/hlc.h"
#include "hlc_kernels.hpp"

namespace hlc {
namespace {

constexpr int MAX_DEVICES = 64;
constexpr double SKY_ARCSEC2 = 5.3458e11;  // 4 pi sr in square arcsec
constexpr double U64 = 1.1102230246251565e-16;
constexpr double ETA64 = 4e-15;             // bound on |chord_fp64 - chord| (unit sphere)

struct Device {
  bool init = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Counters* cnt = nullptr;        // device
  Counters* cnt_host = nullptr;   // pinned host mirror
  hipEvent_t ev[8] = {};
};

Device g_dev[MAX_DEVICES];
hlc_stats g_stats;

int map_err(hipError_t e) {
  if (e == hipSuccess) return HLC_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return HLC_E_NOMEM;
  return HLC_E_DEVICE;
}

#define HLC_TRY(x)                 \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) return map_err(e_); \
  } while (0)

int get_device(Device** out) {
  int dev = 0;
  HLC_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return HLC_E_DEVICE;
  Device& d = g_dev[dev];
  if (!d.init) {
    HLC_TRY(hipMalloc(&d.cnt, sizeof(Counters)));
    HLC_TRY(hipHostMalloc(&d.cnt_host, sizeof(Counters), hipHostMallocDefault));
    for (auto& e : d.ev) HLC_TRY(hipEventCreate(&e));
    d.init = true;
  }
  *out = &d;
  return HLC_OK;
}

// Bump allocator over the device workspace.
struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += n * sizeof(T);
    return p;
  }
};

int ensure_ws(Device& d, size_t bytes) {
  if (bytes <= d.ws_bytes) return HLC_OK;
  if (d.ws) {
    hipDeviceSynchronize();
    hipFree(d.ws);
    d.ws = nullptr;
    d.ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4 + (1 << 20);
  if (const char* f = std::getenv("HLC_TEST_FAIL_ALLOC")) {
    if (std::atoll(f) > 0 && want >= (size_t)std::atoll(f)) return HLC_E_NOMEM;
  }
  hipError_t e = hipMalloc(&d.ws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    d.ws = nullptr;
    return HLC_E_NOMEM;
  }
  d.ws_bytes = want;
  return HLC_OK;
}

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

// Partition geometry for radius r and the catalogue sizes.
Geom make_geom(double r_arcsec, int64_t na, int64_t nb, const hlc_tuning* tu) {
  Geom g;
  g.r_deg = r_arcsec / 3600.0;
  g.rpad_deg = g.r_deg * (1.0 + 1e-9) + 1e-12;
  double h_as;
  if (tu && tu->zone_height_arcsec > 0) {
    h_as = tu->zone_height_arcsec;
  } else {
    // Zone height balancing Dec and RA overhead for a uniform sky of this
    // density: h = sqrt(GROUP / density).
    double rho = (double)std::max<int64_t>(1, std::max(na, nb)) / SKY_ARCSEC2;
    h_as = std::sqrt((double)GROUP / rho);
    h_as = std::min(std::max(h_as, 8.0 * r_arcsec), 3600.0);
  }
  double h = h_as / 3600.0;
  h = std::max(h, 2.0001 * g.rpad_deg);
  h = std::max(h, 180.0 / 65536.0);
  int64_t nz = (int64_t)std::ceil(180.0 / h);
  if (nz < 1) nz = 1;
  g.h_deg = h;
  g.inv_h = 1.0 / h;
  g.nz = (int32_t)nz;
  int zb = ceil_log2((uint64_t)nz);
  g.rb = std::min(30, 32 - zb);
  g.nbins = 1u << g.rb;
  g.bin_scale = (double)g.nbins / 360.0;
  // FP32 cells: RA extent comparable to the zone height
  int sb = 0;
  int shift_override = tu ? tu->ra_cell_bins_log2 : 0;
  if (shift_override > 0) {
    sb = std::max(0, g.rb - shift_override);
  } else {
    double want = 360.0 / h;
    sb = std::min(std::max(0, (int)std::lround(std::log2(std::max(1.0, want)))), std::min(g.rb, 20));
  }
  g.cell_shift = g.rb - sb;
  g.nsuper = 1u << sb;
  g.pad_ = 0;
  return g;
}

struct Plan {
  Geom g;
  int key_bits;
  uint32_t na, nb, nb2;
  double c_r, t_lo64, t_hi64, H_lo, H_hi;
  bool fp32;
};

void thresholds(Plan& p, double r_arcsec) {
  const double r_rad = (r_arcsec / 3600.0) * (M_PI / 180.0);
  const double s = std::sin(0.5 * r_rad);
  p.c_r = 2.0 * s;
  double hi = p.c_r * (1.0 + 4.0 * U64) + ETA64;
  p.t_hi64 = hi * hi * (1.0 + 4.0 * U64);
  double lo = p.c_r * (1.0 - 4.0 * U64) - ETA64;
  p.t_lo64 = lo > 0 ? lo * lo * (1.0 - 4.0 * U64) : -1.0;
  const double H = s * s;
  p.H_lo = H * (1.0 - EPS_BAND);
  p.H_hi = H * (1.0 + EPS_BAND);
}

int check_common(double r_arcsec, int64_t na, int64_t nb, const hlc_opts* o) {
  if (!o || !o->n_pairs) return HLC_E_INVAL;
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return HLC_E_INVAL;
  if (na < 0 || nb < 0 || na >= (int64_t(1) << 31) || nb >= (int64_t(1) << 31)) return HLC_E_INVAL;
  if (o->capacity < 0) return HLC_E_INVAL;
  if (o->precision != HLC_FP32_RECHECK && o->precision != HLC_FP64) return HLC_E_INVAL;
  if (o->flags & HLC_SORTED) return HLC_E_UNSUPPORTED;
  return HLC_OK;
}

struct Bufs {
  uint32_t *kA, *vA, *kB, *vB, *kAlt, *vAlt, *counts, *bsums, *lb, *zstartB;
  int32_t* zmarg;
  double2 *zone_cs, *super_cs;
  GroupRanges* ranges;
  Rec64 *rA64, *rB64;
  Rec32 *rA32, *rB32;
  double2 *radecA, *radecB;
  uint2* band;
};

size_t carve(Carve& c, Bufs& b, const Plan& p, uint64_t band_cap) {
  const uint32_t nA = std::max(p.na, 1u), nB2 = std::max(p.nb2, 1u);
  const uint32_t nmax = std::max(nA, nB2);
  b.kA = c.take<uint32_t>(nA);
  b.vA = c.take<uint32_t>(nA);
  b.kB = c.take<uint32_t>(nB2);
  b.vB = c.take<uint32_t>(nB2);
  b.kAlt = c.take<uint32_t>(nmax);
  b.vAlt = c.take<uint32_t>(nmax);
  b.counts = c.take<uint32_t>(sort_counts_len(nmax));
  b.bsums = c.take<uint32_t>(sort_block_sums_len(nmax));
  b.lb = c.take<uint32_t>(nA);
  b.zstartB = c.take<uint32_t>((size_t)p.g.nz + 1);
  b.zmarg = c.take<int32_t>((size_t)p.g.nz);
  b.zone_cs = c.take<double2>((size_t)p.g.nz);
  b.super_cs = c.take<double2>(p.fp32 ? (size_t)p.g.nsuper : 1);
  b.ranges = c.take<GroupRanges>((nA + GROUP - 1) / GROUP);
  if (p.fp32) {
    b.rA32 = c.take<Rec32>(nA);
    b.rB32 = c.take<Rec32>(nB2);
    b.radecA = c.take<double2>(nA);
    b.radecB = c.take<double2>(nB2);
    b.rA64 = b.rB64 = nullptr;
  } else {
    b.rA64 = c.take<Rec64>(nA);
    b.rB64 = c.take<Rec64>(nB2);
    b.rA32 = b.rB32 = nullptr;
    b.radecA = b.radecB = nullptr;
  }
  b.band = c.take<uint2>(band_cap);
  return c.off + 256;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  hipEventElapsedTime(&ms, a, b);
  return ms;
}

int xmatch_impl(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                double* out_sep, const hlc_opts* o, uint64_t band_cap, bool* retry_band) {
  *retry_band = false;
  Device* dev = nullptr;
  int st = get_device(&dev);
  if (st) return st;
  hipStream_t s = (hipStream_t)o->stream;
  const bool prof = (o->flags & HLC_PROFILE) != 0;
  const bool want_sep = (o->flags & HLC_NO_SEP) == 0;

  Plan p;
  p.fp32 = o->precision == HLC_FP32_RECHECK;
  p.g = make_geom(r_arcsec, na, nb, o->tuning);
  p.na = (uint32_t)na;
  p.nb = (uint32_t)nb;
  p.nb2 = (uint32_t)(2 * nb);
  p.key_bits = ceil_log2((uint64_t)p.g.nz) + p.g.rb;
  thresholds(p, r_arcsec);

  Bufs b;
  Carve sizing{nullptr};
  size_t need = carve(sizing, b, p, band_cap);
  st = ensure_ws(*dev, need);
  if (st) return st;
  Carve c{(char*)dev->ws};
  carve(c, b, p, band_cap);

  Counters* cnt = dev->cnt;
  if (prof) HLC_TRY(hipEventRecord(dev->ev[0], s));
  launch_zero_counters(cnt, s);
  launch_keygen(a_ra, a_dec, p.na, p.g, false, 1u, b.kA, b.vA, cnt, s);
  launch_keygen(b_ra, b_dec, p.nb, p.g, true, 2u, b.kB, b.vB, cnt, s);
  HLC_TRY(hipMemcpyAsync(dev->cnt_host, cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
  if (prof) HLC_TRY(hipEventRecord(dev->ev[1], s));
  HLC_TRY(hipStreamSynchronize(s));
  if (dev->cnt_host->err) {
    *o->n_pairs = 0;
    return HLC_E_INVAL;
  }
  const uint32_t nbh = p.nb + (uint32_t)dev->cnt_host->n_halo;

  SortScratch sc{b.kAlt, b.vAlt, b.counts, b.bsums};
  radix_sort(b.kA, b.vA, p.na, p.key_bits, sc, s);
  radix_sort(b.kB, b.vB, nbh, p.key_bits, sc, s);
  if (prof) HLC_TRY(hipEventRecord(dev->ev[2], s));

  launch_zone_tables(p.g, b.zmarg, b.zone_cs, p.fp32 ? b.super_cs : nullptr, s);
  launch_zone_starts(b.kB, nbh, p.g, b.zstartB, s);
  if (p.fp32) {
    launch_layout32(b.kA, b.vA, p.na, a_ra, a_dec, p.g, b.zone_cs, b.super_cs, b.rA32, b.radecA, s);
    launch_layout32(b.kB, b.vB, nbh, b_ra, b_dec, p.g, b.zone_cs, b.super_cs, b.rB32, b.radecB, s);
  } else {
    launch_layout64(b.vA, p.na, a_ra, a_dec, b.rA64, s);
    launch_layout64(b.vB, nbh, b_ra, b_dec, b.rB64, s);
  }
  if (prof) HLC_TRY(hipEventRecord(dev->ev[3], s));
  launch_merge_lb(b.kA, p.na, b.kB, nbh, b.lb, s);
  launch_ranges(b.kA, p.na, b.lb, b.kB, nbh, b.zstartB, b.zmarg, p.g, p.c_r, b.ranges, s);
  if (prof) HLC_TRY(hipEventRecord(dev->ev[4], s));

  MatchArgs ma{};
  ma.ranges = b.ranges;
  ma.na = p.na;
  ma.nb = nbh;
  ma.recA64 = b.rA64;
  ma.recB64 = b.rB64;
  ma.t_lo64 = p.t_lo64;
  ma.t_hi64 = p.t_hi64;
  ma.recA32 = b.rA32;
  ma.recB32 = b.rB32;
  ma.radecA = b.radecA;
  ma.radecB = b.radecB;
  ma.keysA = b.kA;
  ma.keysB = b.kB;
  ma.zone_cs = b.zone_cs;
  ma.super_cs = b.super_cs;
  ma.geom = p.g;
  ma.H_lo = p.H_lo;
  ma.H_hi = p.H_hi;
  ma.skip_halo_a = 0;
  OutArgs oa{};
  oa.pairs = reinterpret_cast<uint2*>(out_pairs);
  oa.sep = want_sep ? out_sep : nullptr;
  oa.cap = (unsigned long long)o->capacity;
  oa.band = b.band;
  oa.band_cap = band_cap;
  oa.cnt = cnt;
  if (p.fp32) launch_match32(ma, oa, s);
  else launch_match64(ma, oa, s);
  if (prof) HLC_TRY(hipEventRecord(dev->ev[5], s));
  launch_certify(a_ra, a_dec, b_ra, b_dec, r_arcsec, p.H_lo, p.H_hi, oa, s);
  if (prof) HLC_TRY(hipEventRecord(dev->ev[6], s));
  HLC_TRY(hipMemcpyAsync(dev->cnt_host, cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
  if (prof) HLC_TRY(hipEventRecord(dev->ev[7], s));
  HLC_TRY(hipStreamSynchronize(s));
  HLC_TRY(hipGetLastError());

  const Counters& h = *dev->cnt_host;
  if (h.n_band > band_cap) {
    *retry_band = true;
    return HLC_OK;
  }
  std::memset(&g_stats, 0, sizeof(g_stats));
  g_stats.na = na;
  g_stats.nb = nb;
  g_stats.nb_halo = nbh;
  g_stats.n_pairs = (int64_t)h.n_pairs;
  g_stats.n_candidates = (int64_t)h.n_cand;
  g_stats.n_band = (int64_t)h.n_band;
  g_stats.n_ties = (int64_t)h.n_ties;
  g_stats.n_zones = p.g.nz;
  g_stats.ra_bits = p.g.rb;
  g_stats.zone_height_arcsec = p.g.h_deg * 3600.0;
  if (prof) {
    g_stats.t_keygen_ms = elapsed(dev->ev[0], dev->ev[1]);
    g_stats.t_sort_ms = elapsed(dev->ev[1], dev->ev[2]);
    g_stats.t_layout_ms = elapsed(dev->ev[2], dev->ev[3]);
    g_stats.t_ranges_ms = elapsed(dev->ev[3], dev->ev[4]);
    g_stats.t_match_ms = elapsed(dev->ev[4], dev->ev[5]);
    g_stats.t_certify_ms = elapsed(dev->ev[5], dev->ev[6]);
    g_stats.t_total_ms = elapsed(dev->ev[0], dev->ev[7]);
  }
  *o->n_pairs = (int64_t)h.n_pairs;
  return h.n_pairs > (unsigned long long)o->capacity ? HLC_E_OVERFLOW : HLC_OK;
}

}  // namespace
}  // namespace hlc

using namespace hlc;

extern "C" {

int hlc_xmatch(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
               const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
               double* out_sep_arcsec, const hlc_opts* opts) {
  int st = check_common(r_arcsec, na, nb, opts);
  if (st) return st;
  if ((na > 0 && (!a_ra || !a_dec)) || (nb > 0 && (!b_ra || !b_dec))) return HLC_E_INVAL;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  try {
    if (na == 0 || nb == 0) {
      // nothing can match; still reject invalid coordinates on the other side
      Device* dev = nullptr;
      st = get_device(&dev);
      if (st) return st;
      hipStream_t s = (hipStream_t)opts->stream;
      Geom g = make_geom(r_arcsec, na, nb, opts->tuning);
      size_t n = (size_t)std::max(na, nb);
      st = ensure_ws(*dev, 8 * n + 1024);
      if (st) return st;
      uint32_t* k = (uint32_t*)dev->ws;
      uint32_t* v = k + n;
      launch_zero_counters(dev->cnt, s);
      if (na) launch_keygen(a_ra, a_dec, (uint32_t)na, g, false, 1u, k, v, dev->cnt, s);
      if (nb) launch_keygen(b_ra, b_dec, (uint32_t)nb, g, false, 2u, k, v, dev->cnt, s);
      HLC_TRY(hipMemcpyAsync(dev->cnt_host, dev->cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
      HLC_TRY(hipStreamSynchronize(s));
      *opts->n_pairs = 0;
      std::memset(&g_stats, 0, sizeof(g_stats));
      g_stats.na = na;
      g_stats.nb = nb;
      return dev->cnt_host->err ? HLC_E_INVAL : HLC_OK;
    }
    uint64_t band_cap = (1u << 20) + (uint64_t)(na + nb) / 64;
    for (int attempt = 0; attempt < 4; ++attempt) {
      bool retry = false;
      st = xmatch_impl(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, out_pairs, out_sep_arcsec, opts,
                       band_cap, &retry);
      if (!retry) return st;
      band_cap = (uint64_t)(g_dev[0].cnt_host ? 0 : 0) + band_cap * 8;
    }
    return HLC_E_NOMEM;
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

int hlc_partition(const double*, const double*, int64_t, double, const hlc_opts*, struct hlc_part** out) {
  if (out) *out = nullptr;
  return HLC_E_UNSUPPORTED;
}

void hlc_part_free(struct hlc_part*) {}

int hlc_xmatch_part(const struct hlc_part*, const struct hlc_part*, double, hlc_pair*, double*,
                    const hlc_opts*) {
  return HLC_E_UNSUPPORTED;
}

int hlc_xmatch_batch(const hlc_job*, int32_t, const double*, const double*, const double*,
                     const double*, hlc_pair*, double*, int64_t*, const hlc_opts*) {
  return HLC_E_UNSUPPORTED;
}

int hlc_xmatch_stream(const double*, const double*, int64_t, const double*, const double*, int64_t,
                      double, hlc_sink, void*, const hlc_opts*) {
  return HLC_E_UNSUPPORTED;
}

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
  for (auto& d : g_dev) {
    if (!d.init) continue;
    if (d.ws) hipFree(d.ws);
    if (d.cnt) hipFree(d.cnt);
    if (d.cnt_host) hipHostFree(d.cnt_host);
    for (auto& e : d.ev)
      if (e) hipEventDestroy(e);
    d = Device();
  }
}

}  // extern "C"
