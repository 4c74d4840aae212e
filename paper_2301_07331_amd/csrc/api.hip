// api.hip -- the C ABI of libhlc: argument checks, partition geometry,
// per-device workspace, and the order of kernel launches for one call.
//
// A call has two phases that the entry points share:
//   partition(): keygen -> radix sort -> working layout of ONE catalogue
//                (section 4.2's first-level partition, on the GPU);
//   match():     B zone tables -> merge-path lower bounds -> group ranges ->
//                match kernel -> band certification (section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../../include/hlc.h"
#include "hlc_kernels.hpp"

struct hlc_part;

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
  hipEvent_t ev[12] = {};
};

Device g_dev[MAX_DEVICES];
hlc_stats g_stats;

int map_err(hipError_t e) {
  if (e == hipSuccess) return HLC_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return HLC_E_NOMEM;
  return HLC_E_DEVICE;
}

#define HLC_TRY(x)                            \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return map_err(e_); \
  } while (0)

#define HLC_CHECK(x)          \
  do {                        \
    int s_ = (x);             \
    if (s_ != HLC_OK) return s_; \
  } while (0)

int get_device(Device** out, int* dev_id = nullptr) {
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

// Bump allocator over a device buffer (base == nullptr: sizing pass).
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

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

void set_radius(Geom& g, double r_arcsec) {
  g.r_deg = r_arcsec / 3600.0;
  g.rpad_deg = g.r_deg * (1.0 + 1e-9) + 1e-12;
}

// Partition geometry: zone height h_as (arcsec; <= 0 = automatic from the
// catalogue sizes), radius r (halo and windows).
Geom make_geom(double r_arcsec, double h_as, int64_t na, int64_t nb, int cell_log2) {
  Geom g;
  set_radius(g, r_arcsec);
  if (!(h_as > 0)) {
    // zone height balancing Dec and RA overhead for a uniform sky of this
    // density: h = sqrt(GROUP / density)
    double rho = (double)std::max<int64_t>(1, std::max(na, nb)) / SKY_ARCSEC2;
    h_as = std::sqrt((double)GROUP / rho);
    h_as = std::min(std::max(h_as, 8.0 * r_arcsec), 3600.0);
  }
  double h = h_as / 3600.0;
  h = std::max(h, 2.0001 * g.rpad_deg);
  h = std::max(h, 180.0 / 65536.0);
  int64_t nz = std::max<int64_t>(1, (int64_t)std::ceil(180.0 / h));
  g.h_deg = h;
  g.inv_h = 1.0 / h;
  g.nz = (int32_t)nz;
  g.rb = std::min(30, 32 - ceil_log2((uint64_t)nz));
  g.nbins = 1u << g.rb;
  g.bin_scale = (double)g.nbins / 360.0;
  int sb;
  if (cell_log2 > 0) {
    sb = std::max(0, g.rb - cell_log2);
  } else {
    // FP32 cells: RA extent comparable to the zone height
    double want = 360.0 / h;
    sb = std::min(std::max(0, (int)std::lround(std::log2(std::max(1.0, want)))), std::min(g.rb, 20));
  }
  g.cell_shift = g.rb - sb;
  g.nsuper = 1u << sb;
  g.pad_ = 0;
  return g;
}

int key_bits(const Geom& g) { return ceil_log2((uint64_t)g.nz) + g.rb; }

struct Thresholds {
  double c_r, t_lo64, t_hi64, H_lo, H_hi;
};

Thresholds thresholds(double r_arcsec) {
  Thresholds t;
  const double r_rad = (r_arcsec / 3600.0) * (M_PI / 180.0);
  const double s = std::sin(0.5 * r_rad);
  t.c_r = 2.0 * s;
  double hi = t.c_r * (1.0 + 4.0 * U64) + ETA64;
  t.t_hi64 = hi * hi * (1.0 + 4.0 * U64);
  double lo = t.c_r * (1.0 - 4.0 * U64) - ETA64;
  t.t_lo64 = lo > 0 ? lo * lo * (1.0 - 4.0 * U64) : -1.0;
  const double H = s * s;
  t.H_lo = H * (1.0 - EPS_BAND);
  t.H_hi = H * (1.0 + EPS_BAND);
  return t;
}

int check_opts(const hlc_opts* o) {
  if (!o || !o->n_pairs) return HLC_E_INVAL;
  if (o->capacity < 0) return HLC_E_INVAL;
  if (o->precision != HLC_FP32_RECHECK && o->precision != HLC_FP64) return HLC_E_INVAL;
  if (o->flags & HLC_SORTED) return HLC_E_UNSUPPORTED;
  return HLC_OK;
}

int check_common(double r_arcsec, int64_t na, int64_t nb, const hlc_opts* o) {
  HLC_CHECK(check_opts(o));
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return HLC_E_INVAL;
  if (na < 0 || nb < 0 || na >= (int64_t(1) << 31) || nb >= (int64_t(1) << 31)) return HLC_E_INVAL;
  return HLC_OK;
}

double tuned_height(const hlc_opts* o) {
  return (o->tuning && o->tuning->zone_height_arcsec > 0) ? o->tuning->zone_height_arcsec : 0.0;
}
int tuned_cells(const hlc_opts* o) { return o->tuning ? o->tuning->ra_cell_bins_log2 : 0; }

// One partitioned catalogue.
struct Side {
  uint32_t n_src = 0, n = 0;  // sources, entries (halo copies included)
  uint32_t *keys = nullptr, *vals = nullptr;
  Rec64* r64 = nullptr;
  Rec32* r32 = nullptr;
  double2* radec = nullptr;
  const double *ra = nullptr, *dec = nullptr;  // original coordinates (for the band list)
};

struct Tables {
  double2* zone_cs = nullptr;
  double2* super_cs = nullptr;
};

// keygen -> sort -> layout for one catalogue. `cap` entries are available in
// the side's buffers (n, or 2n with a halo). With a halo, the halo count is
// read back (one synchronisation) before sorting.
// Profiling event slots (HLC_PROFILE): per partition, {after keygen,
// before sort, after sort, after layout}; -1 = not recorded.
struct Slots {
  int keygen, sort_begin, sort, layout;
};

void mark(Device& dev, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(dev.ev[slot], s);
}

int partition(Device& dev, const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
              bool l64, bool l32, const Tables& tb, const SortScratch& sc, uint32_t err_bit, Side& sd,
              const Slots& sl, hipStream_t s) {
  sd.n_src = n;
  sd.ra = ra;
  sd.dec = dec;
  launch_keygen(ra, dec, n, g, halo, err_bit, sd.keys, sd.vals, dev.cnt, s);
  mark(dev, sl.keygen, s);
  uint32_t nent = n;
  if (halo) {
    HLC_TRY(hipMemcpyAsync(dev.cnt_host, dev.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HLC_TRY(hipStreamSynchronize(s));
    if (dev.cnt_host->err) return HLC_E_INVAL;
    nent = n + (uint32_t)dev.cnt_host->n_halo;
  }
  sd.n = nent;
  mark(dev, sl.sort_begin, s);
  radix_sort(sd.keys, sd.vals, nent, key_bits(g), sc, s);
  mark(dev, sl.sort, s);
  if (l64) launch_layout64(sd.vals, nent, ra, dec, sd.r64, s);
  if (l32) launch_layout32(sd.keys, sd.vals, nent, ra, dec, g, tb.zone_cs, tb.super_cs, sd.r32, sd.radec, s);
  mark(dev, sl.layout, s);
  return HLC_OK;
}

constexpr Slots NO_SLOTS{-1, -1, -1, -1};

struct MatchWs {
  uint32_t* lb;
  GroupRanges* ranges;
  int32_t* zmarg;
  uint32_t* zstartB;  // nullptr: computed here into zstart_buf
  uint32_t* zstart_buf;
  uint2* band;
  uint64_t band_cap;
};

// Everything after the partition: ranges, match, certification.
void match(Device& dev, const Side& A, const Side& B, const Geom& g, double r_arcsec, bool fp32,
           bool skip_halo_a, bool self_only, const Tables& tb, const MatchWs& w, hlc_pair* out_pairs,
           double* out_sep, uint64_t cap, bool prof, hipStream_t s) {
  Thresholds th = thresholds(r_arcsec);
  launch_zone_tables(g, w.zmarg, tb.zone_cs, nullptr, s);
  const uint32_t* zstart = w.zstartB;
  if (!zstart) {
    launch_zone_starts(B.keys, B.n, g, w.zstart_buf, s);
    zstart = w.zstart_buf;
  }
  launch_merge_lb(A.keys, A.n, B.keys, B.n, w.lb, s);
  launch_ranges(A.keys, A.n, w.lb, B.keys, B.n, zstart, w.zmarg, g, th.c_r, w.ranges, s);
  if (prof) (void)hipEventRecord(dev.ev[8], s);
  MatchArgs ma{};
  ma.ranges = w.ranges;
  ma.na = A.n;
  ma.nb = B.n;
  ma.recA64 = A.r64;
  ma.recB64 = B.r64;
  ma.t_lo64 = th.t_lo64;
  ma.t_hi64 = th.t_hi64;
  ma.recA32 = A.r32;
  ma.recB32 = B.r32;
  ma.radecA = A.radec;
  ma.radecB = B.radec;
  ma.keysA = A.keys;
  ma.keysB = B.keys;
  ma.zone_cs = tb.zone_cs;
  ma.super_cs = tb.super_cs;
  ma.geom = g;
  ma.H_lo = th.H_lo;
  ma.H_hi = th.H_hi;
  ma.skip_halo_a = skip_halo_a ? 1 : 0;
  ma.self_only = self_only ? 1 : 0;
  OutArgs oa{};
  oa.pairs = reinterpret_cast<uint2*>(out_pairs);
  oa.sep = out_sep;
  oa.cap = cap;
  oa.band = w.band;
  oa.band_cap = w.band_cap;
  oa.cnt = dev.cnt;
  if (fp32) launch_match32(ma, oa, s);
  else launch_match64(ma, oa, s);
  if (prof) (void)hipEventRecord(dev.ev[9], s);
  launch_certify(A.ra, A.dec, B.ra, B.dec, r_arcsec, th.H_lo, th.H_hi, oa, s);
  if (prof) (void)hipEventRecord(dev.ev[10], s);
}

size_t carve_match_ws(Carve& c, MatchWs& w, uint32_t na_entries, const Geom& g, uint64_t band_cap,
                      bool need_zstart) {
  const uint32_t nA = std::max(na_entries, 1u);
  w.lb = c.take<uint32_t>(nA);
  w.ranges = c.take<GroupRanges>((nA + GROUP - 1) / GROUP);
  w.zmarg = c.take<int32_t>((size_t)g.nz);
  w.zstart_buf = need_zstart ? c.take<uint32_t>((size_t)g.nz + 1) : nullptr;
  w.zstartB = nullptr;
  w.band = c.take<uint2>(band_cap);
  w.band_cap = band_cap;
  return c.off;
}

void carve_side(Carve& c, Side& sd, uint32_t cap, bool l64, bool l32) {
  cap = std::max(cap, 1u);
  sd.keys = c.take<uint32_t>(cap);
  sd.vals = c.take<uint32_t>(cap);
  sd.r64 = l64 ? c.take<Rec64>(cap) : nullptr;
  sd.r32 = l32 ? c.take<Rec32>(cap) : nullptr;
  sd.radec = l32 ? c.take<double2>(cap) : nullptr;
}

void carve_sort(Carve& c, SortScratch& sc, uint32_t nmax) {
  nmax = std::max(nmax, 1u);
  sc.keys_alt = c.take<uint32_t>(nmax);
  sc.vals_alt = c.take<uint32_t>(nmax);
  sc.counts = c.take<uint32_t>(sort_counts_len(nmax));
  sc.block_sums = c.take<uint32_t>(sort_block_sums_len(nmax));
}

void carve_tables(Carve& c, Tables& tb, const Geom& g, bool l32) {
  tb.zone_cs = c.take<double2>((size_t)g.nz);
  tb.super_cs = l32 ? c.take<double2>((size_t)g.nsuper) : nullptr;
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

// Stage times from the event slots: 0 start; B partition 1-4; A partition
// 5-7 (keygen, sort, layout); 8 ranges; 9 match; 10 certify; 11 end.
void fill_times(Device& dev, bool with_partition) {
  auto el = [&](int a, int b) { return (double)elapsed(dev.ev[a], dev.ev[b]); };
  if (with_partition) {
    g_stats.t_keygen_ms = el(0, 1) + el(4, 5);
    g_stats.t_sort_ms = el(2, 3) + el(5, 6);
    g_stats.t_layout_ms = el(3, 4) + el(6, 7);
    g_stats.t_ranges_ms = el(7, 8);
  } else {
    g_stats.t_ranges_ms = el(0, 8);
  }
  g_stats.t_match_ms = el(8, 9);
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

int xmatch_impl(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                double* out_sep, const hlc_opts* o, uint64_t band_cap, uint64_t* band_needed) {
  *band_needed = 0;
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  hipStream_t s = (hipStream_t)o->stream;
  const bool prof = (o->flags & HLC_PROFILE) != 0;
  const bool fp32 = o->precision == HLC_FP32_RECHECK;
  const bool self = (o->flags & HLC_SELF) != 0;
  const Geom g = make_geom(r_arcsec, tuned_height(o), na, nb, tuned_cells(o));
  const uint32_t nB = (uint32_t)nb;
  // self-match: A's entries are B's (halo copies included)
  const uint32_t nA = self ? 2 * nB : (uint32_t)na;

  Side A, B;
  SortScratch sc;
  Tables tb;
  MatchWs w;
  auto lay = [&](Carve& c) {
    if (!self) carve_side(c, A, nA, !fp32, fp32);
    carve_side(c, B, 2 * nB, !fp32, fp32);
    carve_sort(c, sc, std::max(nA, 2 * nB));
    carve_tables(c, tb, g, fp32);
    carve_match_ws(c, w, nA, g, band_cap, true);
  };
  Carve sizing{nullptr};
  lay(sizing);
  HLC_CHECK(ensure_ws(*dev, sizing.off + 256));
  Carve c{(char*)dev->ws};
  lay(c);

  if (prof) HLC_TRY(hipEventRecord(dev->ev[0], s));
  launch_zero_counters(dev->cnt, s);
  if (fp32) launch_zone_tables(g, w.zmarg, tb.zone_cs, tb.super_cs, s);
  // B first: its halo count is read back before its sort; A's keygen and
  // sort then queue behind it without another synchronisation.
  const Slots slB = prof ? Slots{1, 2, 3, 4} : NO_SLOTS;
  const Slots slA = prof ? Slots{5, -1, 6, 7} : NO_SLOTS;
  HLC_CHECK(partition(*dev, b_ra, b_dec, nB, g, true, !fp32, fp32, tb, sc, 2u, B, slB, s));
  if (self) {
    // one partition serves both roles; its halo copies are skipped as A
    for (int k : {slA.keygen, slA.sort, slA.layout}) mark(*dev, k, s);
    A = B;
  } else {
    HLC_CHECK(partition(*dev, a_ra, a_dec, nA, g, false, !fp32, fp32, tb, sc, 1u, A, slA, s));
  }
  match(*dev, A, B, g, r_arcsec, fp32, self, self, tb, w, out_pairs,
        (o->flags & HLC_NO_SEP) ? nullptr : out_sep, (uint64_t)o->capacity, prof, s);
  HLC_CHECK(read_counters(*dev, s, prof));

  const Counters& h = *dev->cnt_host;
  if (h.err) {
    *o->n_pairs = 0;
    return HLC_E_INVAL;
  }
  if (h.n_band > band_cap) {
    *band_needed = h.n_band;
    return HLC_OK;
  }
  fill_stats(h, na, nb, B.n, g);
  if (prof) fill_times(*dev, true);
  *o->n_pairs = (int64_t)h.n_pairs;
  return h.n_pairs > (unsigned long long)o->capacity ? HLC_E_OVERFLOW : HLC_OK;
}

int validate_only(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                  const double* b_dec, int64_t nb, double r_arcsec, const hlc_opts* o) {
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  hipStream_t s = (hipStream_t)o->stream;
  Geom g = make_geom(r_arcsec, 0.0, na, nb, 0);
  size_t n = (size_t)std::max<int64_t>(1, std::max(na, nb));
  HLC_CHECK(ensure_ws(*dev, 8 * n + 1024));
  uint32_t* k = (uint32_t*)dev->ws;
  uint32_t* v = k + n;
  launch_zero_counters(dev->cnt, s);
  if (na) launch_keygen(a_ra, a_dec, (uint32_t)na, g, false, 1u, k, v, dev->cnt, s);
  if (nb) launch_keygen(b_ra, b_dec, (uint32_t)nb, g, false, 2u, k, v, dev->cnt, s);
  HLC_CHECK(read_counters(*dev, s, false));
  *o->n_pairs = 0;
  std::memset(&g_stats, 0, sizeof(g_stats));
  g_stats.na = na;
  g_stats.nb = nb;
  return dev->cnt_host->err ? HLC_E_INVAL : HLC_OK;
}

}  // namespace
}  // namespace hlc

// A reusable partitioned catalogue (built with a halo so it can serve as
// either side; as A its halo copies are skipped).
struct hlc_part {
  int device = 0;
  hlc::Geom g{};
  double r_build = 0;
  void* mem = nullptr;
  hlc::Side side;
  hlc::Tables tb;
  uint32_t* zstart = nullptr;
  double* ra = nullptr;  // private copies of the coordinates
  double* dec = nullptr;
};

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
  if ((opts->flags & HLC_SELF) && (a_ra != b_ra || a_dec != b_dec || na != nb)) return HLC_E_INVAL;
  try {
    if (na == 0 || nb == 0) return validate_only(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, opts);
    uint64_t band_cap = (1u << 20) + (uint64_t)(na + nb) / 64;
    for (int attempt = 0; attempt < 3; ++attempt) {
      uint64_t need = 0;
      st = xmatch_impl(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, out_pairs, out_sep_arcsec, opts,
                       band_cap, &need);
      if (need == 0) return st;
      band_cap = need + need / 4 + 1024;
    }
    return HLC_E_NOMEM;
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

int hlc_partition(const double* ra_deg, const double* dec_deg, int64_t n, double r_arcsec,
                  const hlc_opts* opts, struct hlc_part** out) {
  if (!out) return HLC_E_INVAL;
  *out = nullptr;
  if (!opts) return HLC_E_INVAL;
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return HLC_E_INVAL;
  if (n < 0 || n >= (int64_t(1) << 31)) return HLC_E_INVAL;
  if (n > 0 && (!ra_deg || !dec_deg)) return HLC_E_INVAL;
  if (opts->flags & HLC_SORTED) return HLC_E_UNSUPPORTED;
  try {
    Device* dev = nullptr;
    int dev_id = 0;
    HLC_CHECK(get_device(&dev, &dev_id));
    hipStream_t s = (hipStream_t)opts->stream;
    // Parts must agree on the geometry without seeing each other, so the
    // automatic zone height depends on the radius only.
    double h_as = tuned_height(opts);
    if (!(h_as > 0)) h_as = std::min(std::max(64.0 * r_arcsec, 32.0), 3600.0);
    auto* p = new hlc_part();
    p->device = dev_id;
    p->r_build = r_arcsec;
    p->g = make_geom(r_arcsec, h_as, n, n, tuned_cells(opts));
    const uint32_t nn = (uint32_t)n, cap = 2 * nn;
    auto lay = [&](Carve& c) {
      carve_side(c, p->side, cap, true, true);
      carve_tables(c, p->tb, p->g, true);
      p->zstart = c.take<uint32_t>((size_t)p->g.nz + 1);
      p->ra = c.take<double>(std::max(nn, 1u));
      p->dec = c.take<double>(std::max(nn, 1u));
    };
    Carve sizing{nullptr};
    lay(sizing);
    int st = dev_alloc(&p->mem, sizing.off + 256);
    if (st) {
      delete p;
      return st;
    }
    Carve c{(char*)p->mem};
    lay(c);
    // sort scratch comes from the shared workspace
    SortScratch sc;
    Carve ss{nullptr};
    carve_sort(ss, sc, std::max(cap, 1u));
    st = ensure_ws(*dev, ss.off + 256);
    if (st) {
      hlc_part_free(p);
      return st;
    }
    Carve cs{(char*)dev->ws};
    carve_sort(cs, sc, std::max(cap, 1u));
    if (nn) {
      HLC_TRY(hipMemcpyAsync(p->ra, ra_deg, (size_t)nn * 8, hipMemcpyDeviceToDevice, s));
      HLC_TRY(hipMemcpyAsync(p->dec, dec_deg, (size_t)nn * 8, hipMemcpyDeviceToDevice, s));
    }
    launch_zero_counters(dev->cnt, s);
    launch_zone_tables(p->g, nullptr, p->tb.zone_cs, p->tb.super_cs, s);
    st = partition(*dev, p->ra, p->dec, nn, p->g, true, true, true, p->tb, sc, 1u, p->side, NO_SLOTS, s);
    if (st == HLC_OK) {
      launch_zone_starts(p->side.keys, p->side.n, p->g, p->zstart, s);
      st = read_counters(*dev, s, false);
    }
    if (st == HLC_OK && dev->cnt_host->err) st = HLC_E_INVAL;
    if (st != HLC_OK) {
      hlc_part_free(p);
      return st;
    }
    *out = p;
    return HLC_OK;
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

void hlc_part_free(struct hlc_part* part) {
  if (!part) return;
  if (part->mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(part->mem);
  }
  delete part;
}

int hlc_xmatch_part(const struct hlc_part* A, const struct hlc_part* B, double r_arcsec,
                    hlc_pair* out_pairs, double* out_sep_arcsec, const hlc_opts* opts) {
  if (!A || !B) return HLC_E_INVAL;
  HLC_CHECK(check_opts(opts));
  if (!(r_arcsec > 0.0) || !(r_arcsec <= B->r_build)) return HLC_E_INVAL;
  if (A->g.h_deg != B->g.h_deg || A->g.rb != B->g.rb || A->g.cell_shift != B->g.cell_shift)
    return HLC_E_INVAL;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  try {
    Device* dev = nullptr;
    int dev_id = 0;
    HLC_CHECK(get_device(&dev, &dev_id));
    if (dev_id != A->device || dev_id != B->device) return HLC_E_INVAL;
    hipStream_t s = (hipStream_t)opts->stream;
    const bool prof = (opts->flags & HLC_PROFILE) != 0;
    const bool fp32 = opts->precision == HLC_FP32_RECHECK;
    Geom g = A->g;
    set_radius(g, r_arcsec);
    if (A->side.n_src == 0 || B->side.n_src == 0) {
      *opts->n_pairs = 0;
      std::memset(&g_stats, 0, sizeof(g_stats));
      return HLC_OK;
    }
    uint64_t band_cap = (1u << 20) + (uint64_t)(A->side.n + B->side.n) / 64;
    for (int attempt = 0; attempt < 3; ++attempt) {
      MatchWs w;
      Carve sizing{nullptr};
      carve_match_ws(sizing, w, A->side.n, g, band_cap, false);
      HLC_CHECK(ensure_ws(*dev, sizing.off + 256));
      Carve c{(char*)dev->ws};
      carve_match_ws(c, w, A->side.n, g, band_cap, false);
      w.zstartB = B->zstart;
      if (prof) HLC_TRY(hipEventRecord(dev->ev[0], s));
      launch_zero_counters(dev->cnt, s);
      match(*dev, A->side, B->side, g, r_arcsec, fp32, true, false, A->tb, w, out_pairs,
            (opts->flags & HLC_NO_SEP) ? nullptr : out_sep_arcsec, (uint64_t)opts->capacity, prof, s);
      HLC_CHECK(read_counters(*dev, s, prof));
      const Counters& h = *dev->cnt_host;
      if (h.n_band > band_cap) {
        band_cap = h.n_band + h.n_band / 4 + 1024;
        continue;
      }
      fill_stats(h, A->side.n_src, B->side.n_src, B->side.n, g);
      if (prof) fill_times(*dev, false);
      *opts->n_pairs = (int64_t)h.n_pairs;
      return h.n_pairs > (unsigned long long)opts->capacity ? HLC_E_OVERFLOW : HLC_OK;
    }
    return HLC_E_NOMEM;
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
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
    if (d.ws) (void)hipFree(d.ws);
    if (d.cnt) (void)hipFree(d.cnt);
    if (d.cnt_host) (void)hipHostFree(d.cnt_host);
    for (auto& e : d.ev)
      if (e) (void)hipEventDestroy(e);
    d = Device();
  }
}

}  // extern "C"
