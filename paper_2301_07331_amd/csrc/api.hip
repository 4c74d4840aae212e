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
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hlc.h"
#include "hlc_kernels.hpp"

struct hlc_part;

namespace hlc {
namespace {

constexpr int MAX_DEVICES = 64;
constexpr double U64 = 1.1102230246251565e-16;
constexpr double ETA64 = 4e-15;             // bound on |chord_fp64 - chord| (unit sphere)

struct Device {
  bool init = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Counters* cnt = nullptr;        // device
  Counters* cnt_host = nullptr;   // pinned host mirror
  hipEvent_t ev[15] = {};
  // streaming form: device and pinned host arenas kept between calls
  // (grow-only; released by hlc_shutdown)
  void* sarena[2] = {nullptr, nullptr};
  size_t sarena_bytes[2] = {0, 0};
  void* harena = nullptr;
  size_t harena_bytes = 0;
  // A's partition runs on `side` beside B's on the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr;
  // B sorted (the ranges start) and ranges done (the filter may start)
  hipEvent_t bsorted = nullptr, prepped = nullptr;
  // staging sizes that earlier calls needed (grow-only), so a repeated
  // workload does not pay the overflow re-run again
  uint64_t hint_stage = 0, hint_cand = 0;
  int ncu = 0;  // compute units (persistent grids)
  bool last_full = true;  // the last call's frame was the whole sphere
  // the footprint sample's result, written by the kernel into mapped host
  // memory (4 values, then the call's sequence number) and polled
  unsigned long long* fmsg_host = nullptr;
  unsigned long long* fmsg_dev = nullptr;
  unsigned long long fseq = 0;
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

int zone_bits(int64_t nz) { return std::max(1, ceil_log2((uint64_t)nz)); }

void set_radius(Geom& g, double r_arcsec) {
  g.r_deg = r_arcsec / 3600.0;
  g.rpad_deg = g.r_deg * (1.0 + 1e-9) + 1e-12;
}

// The region the zones and RA bins cover: the whole sphere, or a box around
// the data (every valid source inside it; an RA span under 180 deg, so no
// pair crosses the box's RA edges).
struct Frame {
  bool full_ra = true;
  double dec_lo = -90.0, dec_hi = 90.0;
  double ra_lo = 0.0, ra_span = 360.0;
};

// Smallest value >= v with at most 21 significant bits: b * (v / 2^rb) with
// b < 2^32 is then exact in FP64.
double round_up_21(double v) {
  int e = 0;
  const double m = std::frexp(v, &e);
  return std::ldexp(std::ceil(std::ldexp(m, 20)), e - 20);
}

// Partition geometry: zone height h_as (arcsec; <= 0 = automatic from the
// data density), radius r (halo and windows), frame f.
Geom make_geom(double r_arcsec, double h_as, int64_t na, int64_t nb, int ra_bits, const Frame& f = Frame{}) {
  Geom g;
  set_radius(g, r_arcsec);
  const double dspan = std::max(f.dec_hi - f.dec_lo, 1e-9);
  if (!(h_as > 0)) {
    // zone height balancing Dec and RA overhead for a uniform density over
    // the frame: h = sqrt(GROUP / density)
    const double d2r = M_PI / 180.0, as_per_rad = 648000.0 / M_PI;
    const double area_sr = std::max(std::sin(f.dec_hi * d2r) - std::sin(f.dec_lo * d2r), 1e-18) *
                           std::max(f.ra_span * d2r, 1e-18);
    const double rho = (double)std::max<int64_t>(1, std::max(na, nb)) / (area_sr * as_per_rad * as_per_rad);
    h_as = std::sqrt((double)GROUP / rho);
    h_as = std::min(std::max(h_as, 8.0 * r_arcsec), 3600.0);
  }
  double h = h_as / 3600.0;
  h = std::max(h, 2.0001 * g.rpad_deg);
  h = std::max(h, dspan / 65536.0);
  int64_t nz = std::max<int64_t>(1, (int64_t)std::ceil(dspan / h));
  g.dec0 = f.dec_lo;
  g.dec_s = f.dec_lo;
  g.dec_n = f.dec_hi;
  g.nzs = g.nzn = 0;
  // Polar cap bands: a zone that reaches a pole is scanned as a whole ring,
  // so within 1 deg of a pole the zones are about 16 r high (at least
  // 2.0001 r padded, at most 4096 per band); the zones between keep height
  // h, widened to a whole number of zones.
  const double cap = 1.0;
  const double hc = std::max(std::max(16.0 * g.r_deg, 2.0001 * g.rpad_deg), cap / 4096.0);
  int64_t nzs = 0, nzn = 0;
  double mid_lo = f.dec_lo, mid_hi = f.dec_hi;
  if (hc < h && f.dec_lo < -90.0 + cap) {
    nzs = (int64_t)std::ceil((std::min(-90.0 + cap, f.dec_hi) - f.dec_lo) / hc);
    mid_lo = f.dec_lo + (double)nzs * hc;
  }
  if (hc < h && f.dec_hi > 90.0 - cap) {
    mid_hi = std::max(90.0 - cap, mid_lo);
    nzn = (int64_t)std::ceil((f.dec_hi - mid_hi) / hc);
  }
  const int64_t nzm = (nzs || nzn) ? std::max<int64_t>(1, (int64_t)std::floor((mid_hi - mid_lo) / h)) : 0;
  // (at most 65536 zones in all, as without the bands)
  if ((nzs || nzn) && mid_hi - mid_lo >= h && nzs + nzm + nzn <= 65536) {
    h = (mid_hi - mid_lo) / (double)nzm;
    nz = nzs + nzm + nzn;
    g.dec_s = mid_lo;
    g.dec_n = mid_hi;
    g.nzs = (int32_t)nzs;
    g.nzn = (int32_t)nzn;
  }
  g.hc_deg = g.nzs || g.nzn ? hc : h;
  g.inv_hc = 1.0 / g.hc_deg;
  g.h_deg = h;
  g.inv_h = 1.0 / h;
  g.nz = (int32_t)nz;
  // at least one zone bit: the shift by rb + fb that extracts the zone must
  // stay below 32
  const int zb = zone_bits(nz);
  const int rb_max = std::min(30, 32 - zb);
  const double span = f.full_ra ? 360.0 : round_up_21(std::max(f.ra_span, 1e-9));
  if (ra_bits > 0) {
    g.rb = std::min(ra_bits, rb_max);
  } else {
    // bins about h/8 wide at the equator keep the RA windows tight; the key
    // then takes every bit of the 8-bit radix digits it needs anyway
    int need = (int)std::ceil(std::log2(span * 8.0 / h));
    need = std::min(std::max(need, 1), rb_max);
    const int digits = (zb + need + 7) / 8;
    g.rb = std::min(8 * digits - zb, rb_max);
  }
  g.nbins = 1u << g.rb;
  g.full_ra = f.full_ra ? 1 : 0;
  g.ra0 = f.full_ra ? 0.0 : f.ra_lo;
  g.ra_width = std::ldexp(span, -g.rb);  // exact
  g.bin_scale = (double)g.nbins / span;
  // spare low key bits carry the RA position inside the bin
  g.fb = std::min(8, std::max(0, 32 - zb - g.rb));
  g.frac_sorted = 0;
  return g;
}

double ext_value(unsigned long long code) {
  double v;
  std::memcpy(&v, &code, 8);
  return v;
}

// The frame of a call's data: a sample of both catalogues first; where its
// box covers over a quarter of the sphere the whole sphere is the frame,
// otherwise one pass over every source gives the exact box. (The partition
// keys then resolve a dense patch as finely as the whole sky.)
// Bounding box of the valid sources from the footprint codes (any: at least
// one valid source).
struct Box {
  bool any;
  double dlo, dhi, rlo, rhi;
};
Box read_box(const Counters& h) {
  Box b;
  b.any = h.ext[1] != 0ull;
  b.dlo = ext_value(~h.ext[0]) - 90.0;
  b.dhi = ext_value(h.ext[1]) - 90.0;
  b.rlo = ext_value(~h.ext[2]);
  b.rhi = ext_value(h.ext[3]);
  return b;
}

// Launches the footprint sample of a call; returns its sequence number for
// frame_finish.
unsigned long long frame_sample(Device& dev, const double* a_ra, const double* a_dec, int64_t na,
                                const double* b_ra, const double* b_dec, int64_t nb, hipStream_t s) {
  const unsigned long long seq = ++dev.fseq;
  launch_extent_sample(a_ra, a_dec, (uint32_t)na, b_ra, b_dec, (uint32_t)nb, dev.cnt, dev.fmsg_dev, seq, s);
  return seq;
}

bool is_full(const Frame& f) { return f.full_ra && f.dec_lo == -90.0 && f.dec_hi == 90.0; }

int frame_finish(Device& dev, unsigned long long seq, const double* a_ra, const double* a_dec, int64_t na,
                 const double* b_ra, const double* b_dec, int64_t nb, hipStream_t s, Frame* out) {
  *out = Frame{};
  Counters* hc = dev.cnt_host;
  auto read_ext = [&]() -> int {
    HLC_TRY(hipMemcpyAsync(hc->ext, dev.cnt->ext, sizeof(hc->ext), hipMemcpyDeviceToHost, s));
    HLC_TRY(hipStreamSynchronize(s));
    return HLC_OK;
  };
  auto box = [&]() { return read_box(*hc); };
  auto quarter_sky = [](const Box& b) {
    const double d2r = M_PI / 180.0;
    return (std::sin(b.dhi * d2r) - std::sin(b.dlo * d2r)) * (b.rhi - b.rlo) * d2r > M_PI;
  };
  // the sample's result is polled in host memory (no stream round trip); a
  // result that does not show up falls back to a stream synchronisation
  {
    volatile unsigned long long* msg = dev.fmsg_host;
    const auto t0 = std::chrono::steady_clock::now();
    while (__atomic_load_n(&dev.fmsg_host[4], __ATOMIC_ACQUIRE) != seq) {
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
        HLC_TRY(hipStreamSynchronize(s));
        HLC_TRY(hipGetLastError());
        if (__atomic_load_n(&dev.fmsg_host[4], __ATOMIC_ACQUIRE) != seq) return HLC_E_DEVICE;
      }
    }
    for (int k = 0; k < 4; ++k) hc->ext[k] = msg[k];
  }
  Box b = box();
  if (!b.any || quarter_sky(b)) return HLC_OK;
  launch_extent(a_ra, a_dec, (uint32_t)na, dev.cnt, s);
  launch_extent(b_ra, b_dec, (uint32_t)nb, dev.cnt, s);
  HLC_CHECK(read_ext());
  b = box();
  // a margin far above the rounding of the codes keeps every source inside
  const double m = 1e-9;
  out->dec_lo = std::max(-90.0, b.dlo - m);
  out->dec_hi = std::min(90.0, b.dhi + m);
  if (b.rhi - b.rlo < 170.0) {
    out->full_ra = false;
    out->ra_lo = b.rlo - m;
    out->ra_span = (b.rhi - b.rlo) + 2.0 * m;
  }
  return HLC_OK;
}

int key_bits(const Geom& g) { return zone_bits(g.nz) + g.rb + g.fb; }

struct Thresholds {
  double c_r, t_lo64, t_hi64, H_lo, H_hi;
  float thr32;
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
  // FP32 filter on FP32 unit vectors: (c_r (1 + 8u) + 3.5 (v + 5u))^2 (1 + 6v),
  // rounded up (the derivation is with the match kernels)
  const double v = 0x1p-24;
  const double c32 = t.c_r * (1.0 + 8.0 * U64) + 3.5 * (v + 5.0 * U64);
  const double T = c32 * c32 * (1.0 + 6.0 * v);
  float Tf = (float)T;
  if ((double)Tf < T) Tf = std::nextafter(Tf, INFINITY);
  t.thr32 = Tf;
  return t;
}

int check_opts(const hlc_opts* o) {
  if (!o || !o->n_pairs) return HLC_E_INVAL;
  if (o->capacity < 0) return HLC_E_INVAL;
  if (o->precision != HLC_FP32_RECHECK && o->precision != HLC_FP64) return HLC_E_INVAL;
  if (o->tuning && (o->tuning->ra_bins_log2 < 0 || o->tuning->ra_bins_log2 > 30)) return HLC_E_INVAL;
  return HLC_OK;
}

// Largest catalogue: B's entries (sources plus halo copies, up to twice the
// sources) and every grid rounded up to whole tiles stay below 2^32.
constexpr int64_t MAX_SOURCES = (int64_t(1) << 31) - (int64_t(1) << 16);

int check_common(double r_arcsec, int64_t na, int64_t nb, const hlc_opts* o) {
  HLC_CHECK(check_opts(o));
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return HLC_E_INVAL;
  if (na < 0 || nb < 0 || na > MAX_SOURCES || nb > MAX_SOURCES) return HLC_E_INVAL;
  return HLC_OK;
}

double tuned_height(const hlc_opts* o) {
  return (o->tuning && o->tuning->zone_height_arcsec > 0) ? o->tuning->zone_height_arcsec : 0.0;
}
int tuned_bins(const hlc_opts* o) { return o->tuning ? o->tuning->ra_bins_log2 : 0; }
bool tuned_fraction_sort(const hlc_opts* o) { return o->tuning && o->tuning->fraction_sort == 1; }
// lowest key bit the radix sort orders: 0 when the sub-bin bits are sorted too
int sort_lo(const Geom& g) { return g.frac_sorted ? 0 : g.fb; }
int tuned_items(const hlc_opts* o) { return (o->tuning && o->tuning->filter_items > 0) ? o->tuning->filter_items : 1; }

// One partitioned catalogue.
struct Side {
  uint32_t n_src = 0, n_cap = 0;  // sources; entry capacity (2 n_src with a halo)
  DevCount cnt{0, 0, nullptr};    // entries, halo copies included (device-side)
  uint32_t *keys = nullptr, *vals = nullptr;
  Rec64* r64 = nullptr;
  Rec32* r32 = nullptr;
  double2* radec = nullptr;
  Rec64* src64 = nullptr;     // per-source records written by the keygen
  SrcRec32* src32 = nullptr;  // (nullptr: the layout gathers (ra, dec))
  const double *ra = nullptr, *dec = nullptr;  // original coordinates (for the band list)
};

// keygen -> sort -> layout for one catalogue. The side's buffers hold n
// entries, or 2n with a halo; the halo count stays on the device (DevCount).
// Profiling event slots (HLC_PROFILE): per partition, {after keygen,
// before sort, after sort, after layout}; -1 = not recorded.
struct Slots {
  int keygen, sort_begin, sort, layout;
};

void mark(Device& dev, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(dev.ev[slot], s);
}

// l64 / l32: the side's records are FP64 / FP32; without a sorted layout
// (sd.r64 / sd.r32 null) the per-source records stay in input order and the
// kernels read them through vals
// Partition of one side in two steps (the keygen can run on another stream
// than the sort): keys (and the per-source records) first, then the sort and
// the sorted layout. sorted_ev (optional) is recorded once the keys are
// sorted, before the records are gathered.
void partition_keys(Device& dev, const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
                    bool l64, bool l32, const SortScratch& sc, uint32_t err_bit, Side& sd, const Slots& sl,
                    hipStream_t s) {
  sd.n_src = n;
  sd.ra = ra;
  sd.dec = dec;
  // an odd number of radix passes ends in the scratch pair unless it starts there
  const bool from_alt = (radix_passes(key_bits(g), sort_lo(g)) & 1) != 0;
  uint32_t* kk = from_alt ? sc.keys_alt : sd.keys;
  uint32_t* vv = from_alt ? sc.vals_alt : sd.vals;
  launch_keygen(ra, dec, n, g, halo, err_bit, kk, vv, dev.cnt, s, l64 ? sd.src64 : nullptr,
                l32 ? sd.src32 : nullptr);
  mark(dev, sl.keygen, s);
  sd.n_cap = halo ? 2 * n : n;
  sd.cnt = halo ? DevCount{n, 2 * n, &dev.cnt->n_halo} : DevCount{n, n, nullptr};
}

int partition_sort(Device& dev, const Geom& g, bool l64, bool l32, const SortScratch& sc, Side& sd,
                   const Slots& sl, hipStream_t s, hipEvent_t sorted_ev = nullptr) {
  const int bits = key_bits(g);
  const bool from_alt = (radix_passes(bits, sort_lo(g)) & 1) != 0;
  mark(dev, sl.sort_begin, s);
  radix_sort(sd.keys, sd.vals, sd.cnt, bits, sc, s, from_alt, sort_lo(g));
  mark(dev, sl.sort, s);
  if (sorted_ev) HLC_TRY(hipEventRecord(sorted_ev, s));
  if (l64 && sd.r64) {
    if (sd.src64) launch_gather64(sd.vals, sd.cnt, sd.src64, sd.r64, s);
    else launch_layout64(sd.vals, sd.cnt, sd.ra, sd.dec, sd.r64, s);
  }
  if (l32 && sd.r32) {
    if (sd.src32) launch_gather32(sd.vals, sd.cnt, sd.src32, sd.r32, sd.radec, s);
    else launch_layout32(sd.vals, sd.cnt, sd.ra, sd.dec, sd.r32, sd.radec, s);
  }
  mark(dev, sl.layout, s);
  return HLC_OK;
}

int partition(Device& dev, const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
              bool l64, bool l32, const SortScratch& sc, uint32_t err_bit, Side& sd,
              const Slots& sl, hipStream_t s, hipEvent_t sorted_ev = nullptr) {
  partition_keys(dev, ra, dec, n, g, halo, l64, l32, sc, err_bit, sd, sl, s);
  return partition_sort(dev, g, l64, l32, sc, sd, sl, s, sorted_ev);
}

constexpr Slots NO_SLOTS{-1, -1, -1, -1};

// Coarse index of B's sorted keys: one entry per 2^shift keys, at most 2^18
struct KeyIndex {
  int shift;
  uint32_t T;
};
// (never finer than the sorted key bits: the low fb bits of a sorted key
// array are in input order within a bin, so the index is exact only on
// multiples of 2^fb)
KeyIndex key_index_dims(const Geom& g) {
  const int kb = key_bits(g);
  const int shift = std::max(std::max(6, kb - 18), sort_lo(g));
  return KeyIndex{shift, (uint32_t)((1ull << std::max(kb - shift, 0)) + 1)};
}

struct MatchWs {
  uint32_t* lb;
  uint32_t* kidx;
  GroupRanges* ranges;
  int32_t* zmarg;
  double* zdelta;
  uint32_t* zstartB;  // nullptr: computed here into zstart_buf
  uint32_t* zstart_buf;
  uint2* band;
  uint64_t band_cap;
  Regions reg;
};

// Sizes of the spill-prone work buffers of a call: the band list, the pair
// slots per output region and the candidate slots per candidate region (0:
// candidates are not staged). All start from estimates; a call whose counts
// exceed them runs again with the counted sizes (the counts are
// deterministic, so the second run fits).
struct Caps {
  uint64_t band;
  uint64_t stage;
  uint64_t cand;
};

uint64_t stage_guess(uint64_t cap) {
  const uint64_t s = cap / NREG + cap / (4 * NREG) + 4096;
  return std::min<uint64_t>(s, 1ull << 22);
}

Caps initial_caps(const Device& d, uint64_t entries, uint64_t cap, bool stage_cand) {
  Caps k;
  k.band = (1u << 20) + entries / 64;
  k.stage = std::max(stage_guess(cap), d.hint_stage);
  k.cand = stage_cand ? std::max(std::min<uint64_t>(entries / (2 * NREG) + 4096, 1ull << 22), d.hint_cand) : 0;
  return k;
}

void carve_regions(Carve& c, Regions& r, const Caps& k, bool sep) {
  r.fill = c.take<unsigned long long>((size_t)NREG * REG_STRIDE);
  r.cfill = c.take<unsigned long long>((size_t)NREG * REG_STRIDE);
  r.S = k.stage;
  r.pairs = c.take<uint2>((size_t)NREG * k.stage);
  r.sep = sep ? c.take<double>((size_t)NREG * k.stage) : nullptr;
  r.Sc = k.cand;
  r.cand = k.cand ? c.take<Cand>((size_t)NREG * k.cand) : nullptr;
  r.cpre = c.take<unsigned long long>((size_t)NREG + 1);
}

// True when the call must run again: its band list overflowed, a candidate
// region overflowed, or a pair region overflowed although the caller's
// buffer holds every pair.
bool regrow(Device& d, const Counters& h, uint64_t cap, Caps& k) {
  bool again = false;
  if (h.n_band > k.band) {
    k.band = h.n_band + h.n_band / 4 + 1024;
    again = true;
  }
  if (k.cand && h.cand_max > k.cand) {
    k.cand = h.cand_max + h.cand_max / 8 + 1024;
    d.hint_cand = std::max(d.hint_cand, k.cand);
    again = true;
  }
  if (!again && h.n_pairs <= cap && h.region_max > k.stage) {
    k.stage = h.region_max + h.region_max / 8 + 1024;
    d.hint_stage = std::max(d.hint_stage, k.stage);
    again = true;
  }
  return again;
}

OutArgs out_args(hlc_pair* pairs, double* sep, uint64_t cap, uint2* band, uint64_t band_cap,
                 const Regions& reg, Counters* cnt) {
  OutArgs oa{};
  oa.pairs = reinterpret_cast<uint2*>(pairs);
  oa.sep = sep;
  oa.cap = cap;
  oa.band = band;
  oa.band_cap = band_cap;
  oa.cnt = cnt;
  oa.reg = reg;
  oa.reg.sep = sep ? reg.sep : nullptr;
  return oa;
}

// Everything after the partition: ranges, match, certification.
void match(Device& dev, const Side& A, const Side& B, const Geom& g, double r_arcsec, bool fp32,
           bool skip_halo_a, bool self_only, const Radii& rad, const MatchWs& w,
           hlc_pair* out_pairs, double* out_sep, uint64_t cap, bool prof, int filter_items, hipStream_t s,
           hipStream_t ps = nullptr) {
  // zone tables, key index and ranges need only the sorted keys: on ps
  // (ordered by the caller after both sorts) they overlap B's gather on s
  if (!ps) ps = s;
  Thresholds th = thresholds(r_arcsec);
  launch_zone_tables(g, w.zmarg, w.zdelta, ps);
  const uint32_t* zstart = w.zstartB;
  if (!zstart) {
    launch_zone_starts(B.keys, B.cnt, g, w.zstart_buf, ps);
    zstart = w.zstart_buf;
  }
  const KeyIndex ki = key_index_dims(g);
  launch_key_index(B.keys, B.cnt, ki.shift, ki.T, w.kidx, ps);
  launch_ranges(A.keys, A.cnt, w.kidx, ki.shift, ki.T, B.keys, zstart, w.zmarg, w.zdelta, g, w.ranges, ps);
  if (prof) (void)hipEventRecord(dev.ev[8], ps);
  // the candidate regions are cleared before the join, beside the ranges
  const OutArgs oa = out_args(out_pairs, out_sep, cap, w.band, w.band_cap, w.reg, dev.cnt);
  launch_regions_reset(oa, s);
  // The filter and what follows run on ps after the ranges, once B's records
  // are gathered on s (that event is usually complete by then, so the join
  // costs no latency); the caller reads the counters on ps.
  hipStream_t ts = s;
  if (ps != s) {
    (void)hipEventRecord(dev.prepped, s);
    (void)hipStreamWaitEvent(ps, dev.prepped, 0);
    ts = ps;
  }
  if (prof) (void)hipEventRecord(dev.ev[13], ts);
  MatchArgs ma{};
  ma.ranges = w.ranges;
  ma.na = A.cnt;
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
  ma.thr32 = th.thr32;
  if (!(fp32 ? (const void*)A.r32 : (const void*)A.r64)) {
    ma.valsA = A.vals;
    ma.srcA64 = A.src64;
    ma.srcA32 = A.src32;
  }
  ma.geom = g;
  ma.H_lo = th.H_lo;
  ma.H_hi = th.H_hi;
  ma.skip_halo_a = skip_halo_a ? 1 : 0;
  ma.self_only = self_only ? 1 : 0;
  ma.a_err = rad.a_err;
  ma.b_err = rad.b_err;
  ma.k_sigma = rad.k;
  ma.hp_order = -1;
  launch_filter(ma, oa, fp32, filter_items, ts);
  if (prof) (void)hipEventRecord(dev.ev[9], ts);
  launch_cand(ma, oa, fp32, ts);
  launch_certify(A.ra, A.dec, B.ra, B.dec, r_arcsec, th.H_lo, th.H_hi, rad, oa, ts);
  launch_compact(oa, ts);
  if (prof) (void)hipEventRecord(dev.ev[10], ts);
}

size_t carve_match_ws(Carve& c, MatchWs& w, uint32_t na_entries, const Geom& g, const Caps& caps,
                      bool need_zstart) {
  const uint64_t band_cap = caps.band;
  const uint32_t nA = std::max(na_entries, 1u);
  w.lb = c.take<uint32_t>(nA);
  w.ranges = c.take<GroupRanges>((nA + GROUP - 1) / GROUP);
  w.zmarg = c.take<int32_t>((size_t)g.nz);
  w.kidx = c.take<uint32_t>(key_index_dims(g).T);
  w.zdelta = c.take<double>((size_t)g.nz);
  w.zstart_buf = need_zstart ? c.take<uint32_t>((size_t)g.nz + 1) : nullptr;
  w.zstartB = nullptr;
  w.band = c.take<uint2>(band_cap);
  w.band_cap = band_cap;
  carve_regions(c, w.reg, caps, true);
  return c.off;
}

// cap entries; n_src > 0 also carves the per-source records of the keygen;
// without `layout` no sorted records are carved (the side is read in place)
void carve_side(Carve& c, Side& sd, uint32_t cap, bool l64, bool l32, uint32_t n_src = 0, bool layout = true) {
  cap = std::max(cap, 1u);
  sd.keys = c.take<uint32_t>(cap);
  sd.vals = c.take<uint32_t>(cap);
  sd.r64 = (l64 && layout) ? c.take<Rec64>(cap) : nullptr;
  sd.r32 = (l32 && layout) ? c.take<Rec32>(cap) : nullptr;
  sd.radec = (l32 && layout) ? c.take<double2>(cap) : nullptr;
  sd.src64 = (l64 && n_src) ? c.take<Rec64>(n_src) : nullptr;
  sd.src32 = (l32 && n_src) ? c.take<SrcRec32>(n_src) : nullptr;
}

void carve_sort(Carve& c, SortScratch& sc, uint32_t nmax) {
  nmax = std::max(nmax, 1u);
  sc.keys_alt = c.take<uint32_t>(nmax);
  sc.vals_alt = c.take<uint32_t>(nmax);
  sc.counts = c.take<uint32_t>(sort_counts_len(nmax));
  sc.digit_totals = c.take<uint32_t>(sort_digit_totals_len(nmax));
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

int xmatch_impl(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                double* out_sep, const hlc_opts* o, Caps& caps, bool* again, const Radii& rad) {
  *again = false;
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  hipStream_t s = (hipStream_t)o->stream;
  const bool prof = (o->flags & HLC_PROFILE) != 0;
  const bool fp32 = o->precision == HLC_FP32_RECHECK;
  const bool self = (o->flags & HLC_SELF) != 0;
  if (prof) HLC_TRY(hipEventRecord(dev->ev[0], s));
  const int64_t na_frame = self ? 0 : na;
  const unsigned long long seq = frame_sample(*dev, a_ra, a_dec, na_frame, b_ra, b_dec, nb, s);
  const uint32_t nB = (uint32_t)nb;
  // self-match: A's entries are B's (halo copies included)
  const uint32_t nA = self ? 2 * nB : (uint32_t)na;
  const Slots slB = prof ? Slots{1, 2, 3, 4} : NO_SLOTS;
  const Slots slA = prof ? Slots{5, -1, 6, 7} : NO_SLOTS;

  Geom g = make_geom(r_arcsec, tuned_height(o), na, nb, tuned_bins(o), Frame{});
  // (set before A's speculative keygen: the number of radix passes decides
  // which buffer that keygen writes)
  g.frac_sorted = tuned_fraction_sort(o) ? 1 : 0;
  Side A, B;
  SortScratch sc, scA;
  MatchWs w;
  auto lay = [&](Carve& c) {
    // A is read in place: the filter gathers its records itself
    if (!self) {
      carve_side(c, A, nA, !fp32, fp32, nA, false);
      carve_sort(c, scA, nA);
    }
    carve_side(c, B, 2 * nB, !fp32, fp32, nB);
    carve_sort(c, sc, 2 * nB);
    carve_match_ws(c, w, nA, g, caps, true);
  };
  // While the host waits for the sample, A's and B's keys under the
  // whole-sphere frame are computed if the previous call on this device had
  // that frame and the workspace already fits it (the places of their
  // buffers do not depend on the frame). They are kept if the sample
  // confirms the frame, else computed again.
  bool spec = false;
  if (!self && dev->last_full) {
    Carve sizing{nullptr};
    lay(sizing);
    if (sizing.off + 256 <= dev->ws_bytes) {
      Carve c{(char*)dev->ws};
      lay(c);
      if (prof) HLC_TRY(hipEventRecord(dev->ev[14], s));
      launch_zero_counters(dev->cnt, s);
      // A's on the side stream, where A's sort follows, B's beside it on the
      // caller's stream (the places of B's buffers do not depend on the frame
      // either)
      HLC_TRY(hipEventRecord(dev->fork, s));
      HLC_TRY(hipStreamWaitEvent(dev->side, dev->fork, 0));
      partition_keys(*dev, a_ra, a_dec, nA, g, false, !fp32, fp32, scA, 1u, A, slA, dev->side);
      partition_keys(*dev, b_ra, b_dec, nB, g, true, !fp32, fp32, sc, 2u, B, slB, s);
      spec = true;
    }
  }
  Frame f;
  HLC_CHECK(frame_finish(*dev, seq, a_ra, a_dec, na_frame, b_ra, b_dec, nb, s, &f));
  dev->last_full = is_full(f);
  const bool keep = spec && dev->last_full;  // the speculative keys stand
  g = make_geom(r_arcsec, tuned_height(o), na, nb, tuned_bins(o), f);
  g.frac_sorted = tuned_fraction_sort(o) ? 1 : 0;
  Carve sizing{nullptr};
  lay(sizing);
  HLC_CHECK(ensure_ws(*dev, sizing.off + 256));
  Carve c{(char*)dev->ws};
  lay(c);

  if (!keep) {
    if (spec) {
      // the speculative keys are dropped: their kernel ends before the
      // counters are cleared again
      HLC_TRY(hipEventRecord(dev->prepped, dev->side));
      HLC_TRY(hipStreamWaitEvent(s, dev->prepped, 0));
    }
    if (prof) HLC_TRY(hipEventRecord(dev->ev[14], s));
    launch_zero_counters(dev->cnt, s);
  }
  // A's partition on the side stream, B's on the caller's, the two keygens
  // side by side; the ranges run on the side stream once both are sorted,
  // beside B's gather (separate sort scratch, disjoint counter fields)
  if (!self) {
    if (!keep) {
      HLC_TRY(hipEventRecord(dev->fork, s));
      HLC_TRY(hipStreamWaitEvent(dev->side, dev->fork, 0));
      partition_keys(*dev, a_ra, a_dec, nA, g, false, !fp32, fp32, scA, 1u, A, slA, dev->side);
    }
  } else {
    mark(*dev, slA.keygen, s);
  }
  if (!keep) partition_keys(*dev, b_ra, b_dec, nB, g, true, !fp32, fp32, sc, 2u, B, slB, s);
  if (!self) HLC_CHECK(partition_sort(*dev, g, !fp32, fp32, scA, A, slA, dev->side));
  HLC_CHECK(partition_sort(*dev, g, !fp32, fp32, sc, B, slB, s, dev->bsorted));
  if (self) {
    // one partition serves both roles; its halo copies are skipped as A
    for (int k : {slA.sort, slA.layout}) mark(*dev, k, s);
    A = B;
  }
  HLC_TRY(hipStreamWaitEvent(dev->side, dev->bsorted, 0));
  mark(*dev, prof ? 12 : -1, dev->side);
  match(*dev, A, B, g, r_arcsec, fp32, self, self, rad, w, out_pairs,
        (o->flags & HLC_NO_SEP) ? nullptr : out_sep, (uint64_t)o->capacity, prof, tuned_items(o), s, dev->side);
  // the match ended on the side stream (after every kernel of the call on s)
  HLC_CHECK(read_counters(*dev, dev->side, prof));

  const Counters& h = *dev->cnt_host;
  if (h.err) {
    *o->n_pairs = 0;
    return HLC_E_INVAL;
  }
  if (regrow(*dev, h, (uint64_t)o->capacity, caps)) {
    *again = true;
    return HLC_OK;
  }
  fill_stats(h, na, nb, nb + (int64_t)h.n_halo, g);
  if (prof) fill_times(*dev, true);
  *o->n_pairs = (int64_t)h.n_pairs;
  return h.n_pairs > (unsigned long long)o->capacity ? HLC_E_OVERFLOW : HLC_OK;
}

// xmatch_impl with the work-buffer retry.
int xmatch_core(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                double* out_sep, const hlc_opts* o, const Radii& rad = Radii{nullptr, nullptr, 0.0}) {
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  Caps caps = initial_caps(*dev, (uint64_t)(na + nb), (uint64_t)o->capacity, true);
  for (int attempt = 0; attempt < 3; ++attempt) {
    bool again = false;
    int st = xmatch_impl(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, out_pairs, out_sep, o, caps, &again, rad);
    if (!again) return st;
  }
  return HLC_E_NOMEM;
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

int bits_for(int64_t n) { return std::max(1, ceil_log2((uint64_t)std::max<int64_t>(n, 2))); }

// HLC_SORTED: the call's pairs, already in the caller's buffers, ordered by
// (a, b) (indices below na and nb).
int sort_output(int st, hlc_pair* pairs, double* sep, const hlc_opts* o, int64_t na, int64_t nb) {
  if (st != HLC_OK || !(o->flags & HLC_SORTED)) return st;
  const int64_t n = *o->n_pairs;
  if (n <= 1) return HLC_OK;
  if (n >= (int64_t(1) << 31)) return HLC_E_UNSUPPORTED;
  if (o->flags & HLC_NO_SEP) sep = nullptr;
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  hipStream_t s = (hipStream_t)o->stream;
  const uint32_t m = (uint32_t)n;
  uint32_t *keys = nullptr, *vals = nullptr;
  uint2* tp = nullptr;
  double* ts = nullptr;
  SortScratch sc;
  auto lay = [&](Carve& c) {
    keys = c.take<uint32_t>(m);
    vals = c.take<uint32_t>(m);
    carve_sort(c, sc, m);
    tp = c.take<uint2>(m);
    ts = sep ? c.take<double>(m) : nullptr;
  };
  Carve sz{nullptr};
  lay(sz);
  HLC_CHECK(ensure_ws(*dev, sz.off + 256));
  Carve c{(char*)dev->ws};
  lay(c);
  sort_pairs(reinterpret_cast<uint2*>(pairs), sep, m, bits_for(na), bits_for(nb), keys, vals, tp, ts, sc, s);
  HLC_TRY(hipStreamSynchronize(s));
  HLC_TRY(hipGetLastError());
  return HLC_OK;
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
    return sort_output(xmatch_core(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, out_pairs, out_sep_arcsec, opts),
                       out_pairs, out_sep_arcsec, opts, na, nb);
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

int hlc_xmatch_radii(const double* a_ra, const double* a_dec, const double* a_err, int64_t na,
                     const double* b_ra, const double* b_dec, const double* b_err, int64_t nb,
                     double k_sigma, hlc_pair* out_pairs, double* out_sep_arcsec, const hlc_opts* opts) {
  int st = check_common(1.0, na, nb, opts);
  if (st) return st;
  if (!(k_sigma > 0.0) || !(k_sigma < 1e300)) return HLC_E_INVAL;
  if ((na > 0 && (!a_ra || !a_dec || !a_err)) || (nb > 0 && (!b_ra || !b_dec || !b_err))) return HLC_E_INVAL;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  if (opts->flags & HLC_SELF) return HLC_E_UNSUPPORTED;
  try {
    if (na == 0 || nb == 0) return validate_only(a_ra, a_dec, na, b_ra, b_dec, nb, 1.0, opts);
    // largest radius: filter radius of the whole call (one read-back)
    Device* dev = nullptr;
    HLC_CHECK(get_device(&dev));
    hipStream_t s = (hipStream_t)opts->stream;
    HLC_CHECK(ensure_ws(*dev, 1024));
    unsigned long long* codes = (unsigned long long*)dev->ws;
    launch_zero_counters(dev->cnt, s);
    launch_zero_u64(codes, 2, s);
    launch_err_max(a_err, (uint32_t)na, codes, dev->cnt, s);
    launch_err_max(b_err, (uint32_t)nb, codes + 1, dev->cnt, s);
    unsigned long long h_codes[2];
    HLC_TRY(hipMemcpyAsync(h_codes, codes, sizeof h_codes, hipMemcpyDeviceToHost, s));
    HLC_CHECK(read_counters(*dev, s, false));
    if (dev->cnt_host->err) return HLC_E_INVAL;
    double ea, eb;
    std::memcpy(&ea, &h_codes[0], 8);
    std::memcpy(&eb, &h_codes[1], 8);
    double rmax = k_sigma * std::sqrt(ea * ea + eb * eb) * (1.0 + 1e-12);
    if (!(rmax <= 3600.0)) return HLC_E_INVAL;
    // all errors zero: only identical positions match; any positive filter
    // radius finds them
    rmax = std::max(rmax, 1e-6);
    return sort_output(xmatch_core(a_ra, a_dec, na, b_ra, b_dec, nb, rmax, out_pairs, out_sep_arcsec, opts,
                                   Radii{a_err, b_err, k_sigma}),
                       out_pairs, out_sep_arcsec, opts, na, nb);
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

int hlc_xmatch_quad(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                    const double* b_dec, int64_t nb, double r_arcsec, int32_t order, hlc_pair* out_pairs,
                    double* out_sep_arcsec, const hlc_opts* opts) {
  int st = check_common(r_arcsec, na, nb, opts);
  if (st) return st;
  if (order < 0 || order > 13) return HLC_E_INVAL;
  if (na >= (int64_t(1) << 28) || nb >= (int64_t(1) << 28)) return HLC_E_INVAL;  // 5 entries each
  if ((na > 0 && (!a_ra || !a_dec)) || (nb > 0 && (!b_ra || !b_dec))) return HLC_E_INVAL;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  if (opts->flags & HLC_SELF) return HLC_E_UNSUPPORTED;
  try {
    if (na == 0 || nb == 0) return validate_only(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, opts);
    Device* dev = nullptr;
    HLC_CHECK(get_device(&dev));
    hipStream_t s = (hipStream_t)opts->stream;
    const uint32_t capA = 5u * (uint32_t)na, capB = 5u * (uint32_t)nb;
    Caps caps = initial_caps(*dev, (uint64_t)capA + capB, (uint64_t)opts->capacity, true);
    for (int attempt = 0; attempt < 3; ++attempt) {
      Side A, B;
      SortScratch sc;
      MatchWs w;
      uint32_t* msplit = nullptr;
      Geom g{};
      set_radius(g, r_arcsec);
      g.rb = 0;  // keys are pixels: a candidate must share the A entry's pixel
      g.nz = 1;
      auto lay = [&](Carve& c) {
        carve_side(c, A, capA, true, true);
        carve_side(c, B, capB, true, true);
        carve_sort(c, sc, std::max(capA, capB));
        carve_match_ws(c, w, capA, g, caps, false);
        msplit = c.take<uint32_t>(merge_splits_len(capA, capB));
      };
      Carve sz{nullptr};
      lay(sz);
      HLC_CHECK(ensure_ws(*dev, sz.off + 256));
      Carve c{(char*)dev->ws};
      lay(c);
      launch_zero_counters(dev->cnt, s);
      const double R = r_arcsec / 3600.0;
      launch_hp_keygen(a_ra, a_dec, (uint32_t)na, order, R, 1u, A.keys, A.vals, &dev->cnt->aux[0], dev->cnt, s);
      launch_hp_keygen(b_ra, b_dec, (uint32_t)nb, order, R, 2u, B.keys, B.vals, &dev->cnt->aux[1], dev->cnt, s);
      A.cnt = DevCount{0, capA, &dev->cnt->aux[0]};
      B.cnt = DevCount{0, capB, &dev->cnt->aux[1]};
      A.ra = a_ra; A.dec = a_dec; B.ra = b_ra; B.dec = b_dec;
      const int kb = 2 * order + 4;  // 12 * 4^order < 2^(2 order + 4)
      radix_sort(A.keys, A.vals, A.cnt, kb, sc, s);
      radix_sort(B.keys, B.vals, B.cnt, kb, sc, s);
      launch_layout64(A.vals, A.cnt, a_ra, a_dec, A.r64, s);
      launch_layout64(B.vals, B.cnt, b_ra, b_dec, B.r64, s);
      launch_radec_gather(A.vals, A.cnt, a_ra, a_dec, A.radec, s);
      launch_radec_gather(B.vals, B.cnt, b_ra, b_dec, B.radec, s);
      launch_merge_lb(A.keys, A.cnt, B.keys, B.cnt, msplit, w.lb, s);
      launch_equal_ranges(A.keys, A.cnt, w.lb, B.keys, B.cnt, w.ranges, s);
      const Thresholds th = thresholds(r_arcsec);
      MatchArgs ma{};
      ma.ranges = w.ranges;
      ma.na = A.cnt;
      ma.recA64 = A.r64;
      ma.recB64 = B.r64;
      ma.t_lo64 = th.t_lo64;
      ma.t_hi64 = th.t_hi64;
      ma.radecA = A.radec;
      ma.radecB = B.radec;
      ma.keysA = A.keys;
      ma.keysB = B.keys;
      ma.geom = g;
      ma.H_lo = th.H_lo;
      ma.H_hi = th.H_hi;
      ma.hp_order = order;
      ma.hp_R = R;
      const OutArgs oa = out_args(out_pairs, (opts->flags & HLC_NO_SEP) ? nullptr : out_sep_arcsec,
                                  (uint64_t)opts->capacity, w.band, w.band_cap, w.reg, dev->cnt);
      launch_regions_reset(oa, s);
      launch_filter(ma, oa, false, 1, s);
      launch_cand(ma, oa, false, s);
      launch_certify(a_ra, a_dec, b_ra, b_dec, r_arcsec, th.H_lo, th.H_hi, Radii{nullptr, nullptr, 0.0}, oa, s);
      launch_compact(oa, s);
      HLC_CHECK(read_counters(*dev, s, false));
      const Counters& h = *dev->cnt_host;
      if (h.err) return HLC_E_INVAL;
      if (regrow(*dev, h, (uint64_t)opts->capacity, caps)) continue;
      std::memset(&g_stats, 0, sizeof(g_stats));
      g_stats.na = na;
      g_stats.nb = nb;
      g_stats.nb_halo = (int64_t)h.aux[1];  // B entries (records with their copies)
      g_stats.n_pairs = (int64_t)h.n_pairs;
      g_stats.n_candidates = (int64_t)h.n_cand;
      g_stats.n_band = (int64_t)h.n_band;
      g_stats.n_ties = (int64_t)h.n_ties;
      *opts->n_pairs = (int64_t)h.n_pairs;
      return sort_output(h.n_pairs > (unsigned long long)opts->capacity ? HLC_E_OVERFLOW : HLC_OK, out_pairs,
                         out_sep_arcsec, opts, na, nb);
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
  if (n < 0 || n > MAX_SOURCES) return HLC_E_INVAL;
  if (n > 0 && (!ra_deg || !dec_deg)) return HLC_E_INVAL;
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
    p->g = make_geom(r_arcsec, h_as, n, n, tuned_bins(opts));
    const uint32_t nn = (uint32_t)n, cap = 2 * nn;
    auto lay = [&](Carve& c) {
      carve_side(c, p->side, cap, true, true);
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
    // sort scratch and the keygen's per-source records come from the shared
    // workspace (the part keeps only the sorted entries)
    SortScratch sc;
    auto scratch = [&](Carve& c) {
      carve_sort(c, sc, std::max(cap, 1u));
      p->side.src64 = c.take<Rec64>(std::max(nn, 1u));
      p->side.src32 = c.take<SrcRec32>(std::max(nn, 1u));
    };
    Carve ss{nullptr};
    scratch(ss);
    st = ensure_ws(*dev, ss.off + 256);
    if (st) {
      hlc_part_free(p);
      return st;
    }
    Carve cs{(char*)dev->ws};
    scratch(cs);
    if (nn) {
      HLC_TRY(hipMemcpyAsync(p->ra, ra_deg, (size_t)nn * 8, hipMemcpyDeviceToDevice, s));
      HLC_TRY(hipMemcpyAsync(p->dec, dec_deg, (size_t)nn * 8, hipMemcpyDeviceToDevice, s));
    }
    launch_zero_counters(dev->cnt, s);
    st = partition(*dev, p->ra, p->dec, nn, p->g, true, true, true, sc, 1u, p->side, NO_SLOTS, s);
    p->side.src64 = nullptr;
    p->side.src32 = nullptr;
    if (st == HLC_OK) {
      launch_zone_starts(p->side.keys, p->side.cnt, p->g, p->zstart, s);
      st = read_counters(*dev, s, false);
    }
    if (st == HLC_OK && dev->cnt_host->err) st = HLC_E_INVAL;
    if (st == HLC_OK) {
      // the entry count is final: keep it on the host side of the part
      const uint32_t ne = nn + (uint32_t)dev->cnt_host->n_halo;
      p->side.cnt = DevCount{ne, ne, nullptr};
    }
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
  if (A->g.h_deg != B->g.h_deg || A->g.rb != B->g.rb || A->g.fb != B->g.fb || A->g.nzs != B->g.nzs ||
      A->g.nzn != B->g.nzn || A->g.hc_deg != B->g.hc_deg || A->g.dec_s != B->g.dec_s)
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
    Caps caps = initial_caps(*dev, (uint64_t)A->side.cnt.cap + B->side.cnt.cap, (uint64_t)opts->capacity, true);
    for (int attempt = 0; attempt < 3; ++attempt) {
      MatchWs w;
      Carve sizing{nullptr};
      carve_match_ws(sizing, w, A->side.cnt.cap, g, caps, false);
      HLC_CHECK(ensure_ws(*dev, sizing.off + 256));
      Carve c{(char*)dev->ws};
      carve_match_ws(c, w, A->side.cnt.cap, g, caps, false);
      w.zstartB = B->zstart;
      if (prof) HLC_TRY(hipEventRecord(dev->ev[0], s));
      launch_zero_counters(dev->cnt, s);
      match(*dev, A->side, B->side, g, r_arcsec, fp32, true, false, Radii{nullptr, nullptr, 0.0}, w,
            out_pairs,
            (opts->flags & HLC_NO_SEP) ? nullptr : out_sep_arcsec, (uint64_t)opts->capacity, prof,
            tuned_items(opts), s);
      HLC_CHECK(read_counters(*dev, s, prof));
      const Counters& h = *dev->cnt_host;
      if (regrow(*dev, h, (uint64_t)opts->capacity, caps)) continue;
      fill_stats(h, A->side.n_src, B->side.n_src, B->side.cnt.cap, g);
      if (prof) fill_times(*dev, false);
      *opts->n_pairs = (int64_t)h.n_pairs;
      return sort_output(h.n_pairs > (unsigned long long)opts->capacity ? HLC_E_OVERFLOW : HLC_OK, out_pairs,
                         out_sep_arcsec, opts, A->side.n_src, B->side.n_src);
    }
    return HLC_E_NOMEM;
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

}  // extern "C"

namespace hlc {
namespace {

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
struct BatchPlan {
  int32_t njobs = 0, lb_bits = 31;
  uint64_t NA = 0, NB = 0;
  uint32_t ztotal = 0;
  std::vector<BatchJob> jobs;
  std::vector<BatchTile> tA, tB;
};

// 64-bit hash of a byte range, eight bytes per step (multiply and xor-shift
// mixing of each word into the state).
uint64_t hash_words(const void* p, size_t n, uint64_t h = 0x9e3779b97f4a7c15ull) {
  const unsigned char* c = (const unsigned char*)p;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, c + i, 8);
    h ^= w;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
  }
  uint64_t w = 0;
  std::memcpy(&w, c + i, n - i);
  h ^= w ^ (uint64_t)n;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 29;
  return h;
}

uint64_t fnv(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

int build_plan(const hlc_job* jobs, int32_t njobs, BatchPlan& P) {
  if (njobs < 0 || njobs > 65536) return HLC_E_INVAL;
  if (njobs > 0 && !jobs) return HLC_E_INVAL;
  P.njobs = njobs;
  P.lb_bits = 32 - std::max(1, ceil_log2((uint64_t)std::max(njobs, 1)));
  P.jobs.resize(njobs);
  uint64_t ea = 0, eb = 0, zo = 0;
  const uint32_t zmax = 1u << (P.lb_bits - 8);
  for (int32_t j = 0; j < njobs; ++j) {
    const hlc_job& J = jobs[j];
    if (J.a_off < 0 || J.na < 0 || J.b_off < 0 || J.nb < 0) return HLC_E_INVAL;
    if (!(J.r_arcsec > 0.0) || !(J.r_arcsec <= 3600.0)) return HLC_E_INVAL;
    if (J.a_off + J.na >= (int64_t(1) << 31) || J.b_off + J.nb >= (int64_t(1) << 31)) return HLC_E_INVAL;
    BatchJob& B = P.jobs[j];
    B.a_off = J.a_off;
    B.na = J.na;
    B.b_off = J.b_off;
    B.nb = J.nb;
    B.r_arcsec = J.r_arcsec;
    const double sh = std::sin(0.5 * (J.r_arcsec / 3600.0) * (M_PI / 180.0));
    B.H_lo = sh * sh * (1.0 - EPS_BAND);
    B.H_hi = sh * sh * (1.0 + EPS_BAND);
    B.a_entry = (uint32_t)ea;
    B.b_entry = (uint32_t)eb;
    // zone budget: enough zones for about 16 sources per zone row, at most 2^(LB-8)
    B.zcap = (uint32_t)std::min<uint64_t>(zmax, 4 + (uint64_t)(J.na + J.nb) / 16);
    B.zoff = (uint32_t)zo;
    zo += B.zcap + 1;
    for (int64_t t = 0; t < J.na; t += BATCH_TILE)
      P.tA.push_back({(uint32_t)j, (uint32_t)(ea + t), (uint32_t)(J.a_off + t),
                      (uint32_t)std::min<int64_t>(BATCH_TILE, J.na - t)});
    for (int64_t t = 0; t < J.nb; t += BATCH_TILE)
      P.tB.push_back({(uint32_t)j, (uint32_t)(eb + t), (uint32_t)(J.b_off + t),
                      (uint32_t)std::min<int64_t>(BATCH_TILE, J.nb - t)});
    ea += J.na;
    eb += J.nb;
    if (ea >= (uint64_t(1) << 30) || eb >= (uint64_t(1) << 30) || zo >= (uint64_t(1) << 31))
      return HLC_E_INVAL;
  }
  P.NA = ea;
  P.NB = eb;
  P.ztotal = (uint32_t)zo;
  return HLC_OK;
}

struct BatchState {  // per device
  void* tables = nullptr;
  size_t tables_bytes = 0;
  uint64_t tables_hash = 0;
  BatchJob* d_jobs = nullptr;
  BatchTile *d_tA = nullptr, *d_tB = nullptr;
  hipStream_t st = nullptr;
  hipStream_t st2 = nullptr;  // A's chain, beside B's
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  hipEvent_t ev_fork[2] = {nullptr, nullptr}, ev_join[2] = {nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  uint64_t graph_key = 0;
  int ncu = 256;
  // the last batch's plan, reused while the caller's job table repeats
  BatchPlan plan;
  uint64_t plan_hash = 0;
  bool plan_ok = false;
};
BatchState g_bstate[MAX_DEVICES];
std::vector<std::pair<std::string, double>> g_tune;
bool g_tune_loaded = false;

void drop_graph(BatchState& B) {
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.exec = nullptr;
  B.graph = nullptr;
  B.graph_key = 0;
}

// Flat {"key": number, ...} JSON cache of tuned factors ($HLC_TUNE_CACHE).
void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("HLC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  std::fclose(f);
  size_t i = 0;
  while (true) {
    size_t a = txt.find('"', i);
    if (a == std::string::npos) break;
    size_t b = txt.find('"', a + 1);
    if (b == std::string::npos) break;
    size_t c = txt.find(':', b);
    if (c == std::string::npos) break;
    double v = std::strtod(txt.c_str() + c + 1, nullptr);
    if (v > 0) g_tune.emplace_back(txt.substr(a + 1, b - a - 1), v);
    i = c + 1;
  }
}

void tune_save() {
  const char* path = std::getenv("HLC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t k = 0; k < g_tune.size(); ++k)
    std::fprintf(f, "  \"%s\": %.6g%s\n", g_tune[k].first.c_str(), g_tune[k].second,
                 k + 1 < g_tune.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
}

struct BatchBufs {
  unsigned long long* bounds;
  JobGeom* geo;
  uint32_t *kA, *vA, *kB, *vB, *lb, *msplit, *zstart, *ckey, *cval;
  int32_t* zmarg;
  GroupRanges* ranges;
  Rec64 *rA64, *rB64;
  Rec32 *rA32, *rB32;
  double2 *radecA, *radecB;
  uint2* band;
  uint32_t* band_job;
  uint64_t band_cap;
  Regions reg;
  unsigned long long* jcount;
  SortScratch sc, scA;
};

void carve_batch(Carve& c, BatchBufs& b, const BatchPlan& P, bool fp32, const Caps& caps, bool own_jcount) {
  const uint64_t band_cap = caps.band;
  const uint32_t NA = std::max<uint32_t>((uint32_t)P.NA, 1), NB2 = std::max<uint32_t>(2 * (uint32_t)P.NB, 1);
  const uint32_t ng = (NA + GROUP - 1) / GROUP;
  b.bounds = c.take<unsigned long long>(4 * (size_t)std::max(P.njobs, 1));
  b.geo = c.take<JobGeom>(std::max(P.njobs, 1));
  b.kA = c.take<uint32_t>(NA);
  b.vA = c.take<uint32_t>(NA);
  b.kB = c.take<uint32_t>(NB2);
  b.vB = c.take<uint32_t>(NB2);
  carve_sort(c, b.sc, std::max(NB2, ng));
  carve_sort(c, b.scA, NA);
  if (fp32) {
    b.rA32 = c.take<Rec32>(NA);
    b.rB32 = c.take<Rec32>(NB2);
    b.radecA = c.take<double2>(NA);
    b.radecB = c.take<double2>(NB2);
    b.rA64 = b.rB64 = nullptr;
  } else {
    b.rA64 = c.take<Rec64>(NA);
    b.rB64 = c.take<Rec64>(NB2);
    b.rA32 = b.rB32 = nullptr;
    b.radecA = b.radecB = nullptr;
  }
  b.lb = c.take<uint32_t>(NA);
  b.msplit = c.take<uint32_t>(merge_splits_len(NA, NB2));
  b.ranges = c.take<GroupRanges>(ng);
  b.ckey = c.take<uint32_t>(ng);
  b.cval = c.take<uint32_t>(ng);
  b.zmarg = c.take<int32_t>(std::max<uint32_t>(P.ztotal, 1));
  b.zstart = c.take<uint32_t>(std::max<uint32_t>(P.ztotal, 1));
  b.band = c.take<uint2>(band_cap);
  b.band_job = c.take<uint32_t>(band_cap);
  b.band_cap = band_cap;
  carve_regions(c, b.reg, caps, true);
  b.jcount = own_jcount ? c.take<unsigned long long>(std::max(P.njobs, 1)) : nullptr;
}

// Every launch of one batched call on stream s, A's chain forked to BS.st2
// and joined back (no host synchronisation, so the sequence can be captured
// into a graph with two branches).
void batch_enqueue(Device& dev, BatchState& BS, const BatchPlan& P, const BatchBufs& b, const double* a_ra,
                   const double* a_dec, const double* b_ra, const double* b_dec, hlc_pair* out_pairs,
                   double* out_sep, uint64_t cap, unsigned long long* jcount, double factor, bool fp32,
                   hipStream_t s) {
  const uint32_t NA = (uint32_t)P.NA, NB = (uint32_t)P.NB;
  hipStream_t s2 = BS.st2;
  auto fork = [&](int k) {
    (void)hipEventRecord(BS.ev_fork[k], s);
    (void)hipStreamWaitEvent(s2, BS.ev_fork[k], 0);
  };
  auto join = [&](int k) {
    (void)hipEventRecord(BS.ev_join[k], s2);
    (void)hipStreamWaitEvent(s, BS.ev_join[k], 0);
  };
  launch_zero_counters(dev.cnt, s);
  launch_zero_u64(jcount, (uint32_t)P.njobs, s);
  launch_job_bounds_init(b.bounds, P.njobs, s);
  fork(0);
  launch_job_bounds(BS.d_tA, (uint32_t)P.tA.size(), BS.d_jobs, a_ra, b_ra, a_ra, a_dec, false, b.bounds,
                    dev.cnt, s2);
  launch_job_bounds(BS.d_tB, (uint32_t)P.tB.size(), BS.d_jobs, a_ra, b_ra, b_ra, b_dec, true, b.bounds,
                    dev.cnt, s);
  join(0);
  launch_job_frames(BS.d_jobs, P.njobs, a_ra, b_ra, b.bounds, P.lb_bits, factor, b.geo, s);
  const DevCount cA{NA, NA, nullptr};
  const DevCount cB{NB, 2 * NB, &dev.cnt->n_halo};
  fork(1);
  launch_batch_keygen(BS.d_tA, (uint32_t)P.tA.size(), b.geo, a_ra, a_dec, P.lb_bits, false, NA, b.kA, b.vA,
                      dev.cnt, s2);
  radix_sort(b.kA, b.vA, cA, 32, b.scA, s2);
  if (fp32) launch_batch_layout32(b.kA, b.vA, cA, a_ra, a_dec, b.geo, P.lb_bits, b.rA32, b.radecA, s2);
  else launch_layout64(b.vA, cA, a_ra, a_dec, b.rA64, s2);
  launch_batch_keygen(BS.d_tB, (uint32_t)P.tB.size(), b.geo, b_ra, b_dec, P.lb_bits, true, NB, b.kB, b.vB,
                      dev.cnt, s);
  radix_sort(b.kB, b.vB, cB, 32, b.sc, s);
  if (fp32) launch_batch_layout32(b.kB, b.vB, cB, b_ra, b_dec, b.geo, P.lb_bits, b.rB32, b.radecB, s);
  else launch_layout64(b.vB, cB, b_ra, b_dec, b.rB64, s);
  launch_batch_zone_tables(b.geo, P.njobs, BS.d_jobs, P.ztotal, P.lb_bits, b.kB, cB, b.zmarg, b.zstart, s);
  join(1);
  launch_merge_lb(b.kA, cA, b.kB, cB, b.msplit, b.lb, s);
  launch_batch_ranges(b.kA, cA, b.lb, b.kB, b.geo, P.lb_bits, b.zmarg, b.zstart, b.ranges, b.ckey, b.cval, s);
  const uint32_t ng = (NA + GROUP - 1) / GROUP;
  radix_sort(b.ckey, b.cval, DevCount{ng, ng, nullptr}, 32, b.sc, s);
  BatchMatchArgs ma{};
  ma.ranges = b.ranges;
  ma.order = b.cval;
  ma.queue = &dev.cnt->queue;
  ma.na = cA;
  ma.keysA = b.kA;
  ma.keysB = b.kB;
  ma.recA64 = b.rA64;
  ma.recB64 = b.rB64;
  ma.recA32 = b.rA32;
  ma.recB32 = b.rB32;
  ma.radecA = b.radecA;
  ma.radecB = b.radecB;
  ma.geo = b.geo;
  ma.lb_bits = P.lb_bits;
  ma.job_count = jcount;
  OutArgs oa = out_args(out_pairs, out_sep, cap, b.band, b.band_cap, b.reg, dev.cnt);
  oa.band_job = b.band_job;
  launch_regions_reset(oa, s);
  // persistent grid: four 256-thread blocks per CU (the LDS queue allows four)
  const uint32_t nblocks = std::max<uint32_t>(1, std::min<uint32_t>(4u * (uint32_t)BS.ncu, (ng + 15) / 16));
  launch_batch_match(ma, oa, fp32, nblocks, s);
  launch_batch_certify(a_ra, a_dec, b_ra, b_dec, BS.d_jobs, oa, jcount, s);
  launch_compact(oa, s);
}

int batch_impl(const hlc_job* jobs, int32_t njobs, const double* a_ra, const double* a_dec,
               const double* b_ra, const double* b_dec, hlc_pair* out_pairs, double* out_sep,
               int64_t* job_pair_count, const hlc_opts* o) {
  if (njobs < 0 || njobs > 65536 || (njobs > 0 && !jobs)) return HLC_E_INVAL;
  int dev_id0 = 0;
  Device* dev0 = nullptr;
  HLC_CHECK(get_device(&dev0, &dev_id0));
  BatchState& BS0 = g_bstate[dev_id0];
  // the plan (job frames' bookkeeping and source tiles) follows from the job
  // table alone: kept while the caller passes the same table again
  const uint64_t jh = hash_words(jobs, sizeof(hlc_job) * (size_t)njobs, (uint64_t)njobs);
  if (!BS0.plan_ok || BS0.plan_hash != jh) {
    BS0.plan_ok = false;
    BS0.plan = BatchPlan();
    HLC_CHECK(build_plan(jobs, njobs, BS0.plan));
    BS0.plan_hash = jh;
    BS0.plan_ok = true;
  }
  const BatchPlan& P = BS0.plan;
  if ((P.NA > 0 && (!a_ra || !a_dec)) || (P.NB > 0 && (!b_ra || !b_dec))) return HLC_E_INVAL;
  std::memset(&g_stats, 0, sizeof(g_stats));
  if (P.NA == 0 || P.NB == 0) {
    // nothing can match; still reject invalid coordinates
    int dev_id = 0;
    Device* dev = nullptr;
    HLC_CHECK(get_device(&dev, &dev_id));
    if (job_pair_count && njobs > 0)
      HLC_TRY(hipMemsetAsync(job_pair_count, 0, sizeof(int64_t) * njobs, (hipStream_t)o->stream));
    for (const hlc_job* J = jobs; J < jobs + njobs; ++J) {
      if (J->na > 0) HLC_CHECK(validate_only(a_ra + J->a_off, a_dec + J->a_off, J->na, nullptr, nullptr, 0, J->r_arcsec, o));
      if (J->nb > 0) HLC_CHECK(validate_only(nullptr, nullptr, 0, b_ra + J->b_off, b_dec + J->b_off, J->nb, J->r_arcsec, o));
    }
    *o->n_pairs = 0;
    return HLC_OK;
  }
  int dev_id = 0;
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev, &dev_id));
  BatchState& BS = g_bstate[dev_id];
  if (!BS.st) {
    HLC_TRY(hipStreamCreate(&BS.st));
    HLC_TRY(hipStreamCreateWithFlags(&BS.st2, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
      HLC_TRY(hipEventCreateWithFlags(&BS.ev_fork[k], hipEventDisableTiming));
      HLC_TRY(hipEventCreateWithFlags(&BS.ev_join[k], hipEventDisableTiming));
    }
    HLC_TRY(hipEventCreateWithFlags(&BS.ev_in, hipEventDisableTiming));
    HLC_TRY(hipEventCreateWithFlags(&BS.ev_out, hipEventDisableTiming));
    HLC_TRY(hipEventCreate(&BS.ev_t0));
    HLC_TRY(hipEventCreate(&BS.ev_t1));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev_id) == hipSuccess && prop.multiProcessorCount > 0)
      BS.ncu = prop.multiProcessorCount;
  }
  hipStream_t us = (hipStream_t)o->stream;
  HLC_TRY(hipEventRecord(BS.ev_in, us));
  HLC_TRY(hipStreamWaitEvent(BS.st, BS.ev_in, 0));
  hipStream_t s = BS.st;
  const bool fp32 = o->precision == HLC_FP32_RECHECK;

  // device copies of the job and tile tables (kept while the batch repeats;
  // they follow from the job table, so its hash identifies them)
  const uint64_t th = jh;
  if (th != BS.tables_hash || !BS.tables) {
    drop_graph(BS);
    Carve sz{nullptr};
    sz.take<BatchJob>(P.jobs.size());
    sz.take<BatchTile>(std::max<size_t>(P.tA.size(), 1));
    sz.take<BatchTile>(std::max<size_t>(P.tB.size(), 1));
    if (sz.off + 256 > BS.tables_bytes) {
      if (BS.tables) {
        (void)hipDeviceSynchronize();
        (void)hipFree(BS.tables);
        BS.tables = nullptr;
        BS.tables_bytes = 0;
      }
      HLC_CHECK(dev_alloc(&BS.tables, sz.off + 256));
      BS.tables_bytes = sz.off + 256;
    }
    Carve c{(char*)BS.tables};
    BS.d_jobs = c.take<BatchJob>(P.jobs.size());
    BS.d_tA = c.take<BatchTile>(std::max<size_t>(P.tA.size(), 1));
    BS.d_tB = c.take<BatchTile>(std::max<size_t>(P.tB.size(), 1));
    HLC_TRY(hipMemcpyAsync(BS.d_jobs, P.jobs.data(), P.jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice, s));
    HLC_TRY(hipMemcpyAsync(BS.d_tA, P.tA.data(), P.tA.size() * sizeof(BatchTile), hipMemcpyHostToDevice, s));
    HLC_TRY(hipMemcpyAsync(BS.d_tB, P.tB.data(), P.tB.size() * sizeof(BatchTile), hipMemcpyHostToDevice, s));
    HLC_TRY(hipStreamSynchronize(s));
    BS.tables_hash = th;
  }

  unsigned long long* jcount = reinterpret_cast<unsigned long long*>(job_pair_count);
  const uint64_t cap = (uint64_t)o->capacity;
  Caps caps = initial_caps(*dev, (uint64_t)(P.NA + P.NB), cap, false);
  double* sep = (o->flags & HLC_NO_SEP) ? nullptr : out_sep;

  // zone-height factor: given, cached, or tuned now (eager timed runs)
  double factor = (o->tuning && o->tuning->zone_height_factor > 0) ? o->tuning->zone_height_factor : 0.0;
  char bucket[128];
  std::snprintf(bucket, sizeof bucket, "batch|%s|j%d|a%d|b%d", fp32 ? "fp32" : "fp64",
                ceil_log2((uint64_t)njobs), ceil_log2(P.NA), ceil_log2(P.NB));
  if (!(factor > 0)) {
    tune_load();
    for (auto& kv : g_tune)
      if (kv.first == bucket) factor = kv.second;
  }
  for (int attempt = 0; attempt < 3; ++attempt) {
    BatchBufs b;
    Carve sz{nullptr};
    carve_batch(sz, b, P, fp32, caps, jcount == nullptr);
    HLC_CHECK(ensure_ws(*dev, sz.off + 256));
    Carve c{(char*)dev->ws};
    carve_batch(c, b, P, fp32, caps, jcount == nullptr);
    unsigned long long* jc = jcount ? jcount : b.jcount;
    if (!(factor > 0)) {
      // autotune: time each candidate on this batch
      drop_graph(BS);
      double best_t = 1e30, best_f = 1.0;
      for (double f : {0.35, 0.7, 1.4, 2.8}) {
        HLC_TRY(hipEventRecord(BS.ev_t0, s));
        batch_enqueue(*dev, BS, P, b, a_ra, a_dec, b_ra, b_dec, out_pairs, sep, cap, jc, f, fp32, s);
        HLC_TRY(hipEventRecord(BS.ev_t1, s));
        HLC_TRY(hipStreamSynchronize(s));
        float ms = 0.f;
        HLC_TRY(hipEventElapsedTime(&ms, BS.ev_t0, BS.ev_t1));
        if (ms < best_t) { best_t = ms; best_f = f; }
      }
      factor = best_f;
      g_tune.emplace_back(bucket, factor);
      tune_save();
    }
    const bool prof = (o->flags & HLC_PROFILE) != 0;
    uint64_t gk = fnv(&th, sizeof th);
    const void* keyp[] = {a_ra, a_dec, b_ra, b_dec, out_pairs, sep, jc, dev->ws, dev->cnt};
    gk = fnv(keyp, sizeof keyp, gk);
    const double keyd[] = {factor, (double)cap, (double)caps.band, (double)caps.stage, (double)fp32,
                           (double)dev->ws_bytes};
    gk = fnv(keyd, sizeof keyd, gk);
    if (BS.exec == nullptr || BS.graph_key != gk) {
      drop_graph(BS);
      HLC_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      batch_enqueue(*dev, BS, P, b, a_ra, a_dec, b_ra, b_dec, out_pairs, sep, cap, jc, factor, fp32, s);
      hipError_t e = hipStreamEndCapture(s, &BS.graph);
      if (e != hipSuccess) {
        BS.graph = nullptr;
        return map_err(e);
      }
      e = hipGraphInstantiate(&BS.exec, BS.graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        drop_graph(BS);
        return map_err(e);
      }
      BS.graph_key = gk;
    }
    if (prof) HLC_TRY(hipEventRecord(BS.ev_t0, s));
    HLC_TRY(hipGraphLaunch(BS.exec, s));
    if (prof) HLC_TRY(hipEventRecord(BS.ev_t1, s));
    HLC_TRY(hipMemcpyAsync(dev->cnt_host, dev->cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HLC_TRY(hipStreamSynchronize(s));
    HLC_TRY(hipEventRecord(BS.ev_out, s));
    HLC_TRY(hipStreamWaitEvent(us, BS.ev_out, 0));
    const Counters& h = *dev->cnt_host;
    if (h.err) {
      *o->n_pairs = 0;
      return HLC_E_INVAL;
    }
    if (regrow(*dev, h, cap, caps)) {
      drop_graph(BS);
      continue;
    }
    g_stats.na = (int64_t)P.NA;
    g_stats.nb = (int64_t)P.NB;
    g_stats.nb_halo = (int64_t)(P.NB + h.n_halo);
    g_stats.n_pairs = (int64_t)h.n_pairs;
    g_stats.n_candidates = (int64_t)h.n_cand;
    g_stats.n_band = (int64_t)h.n_band;
    g_stats.n_ties = (int64_t)h.n_ties;
    g_stats.n_zones = (int32_t)P.ztotal;
    g_stats.zone_height_arcsec = factor;  // batched form: the zone-height factor used
    if (prof) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, BS.ev_t0, BS.ev_t1);
      g_stats.t_total_ms = ms;
    }
    *o->n_pairs = (int64_t)h.n_pairs;
    return h.n_pairs > cap ? HLC_E_OVERFLOW : HLC_OK;
  }
  return HLC_E_NOMEM;
}

}  // namespace
}  // namespace hlc

extern "C" {

int hlc_xmatch_batch(const hlc_job* jobs, int32_t njobs, const double* a_ra, const double* a_dec,
                     const double* b_ra, const double* b_dec, hlc_pair* out_pairs, double* out_sep_arcsec,
                     int64_t* job_pair_count, const hlc_opts* opts) {
  HLC_CHECK(check_opts(opts));
  if (opts->flags & HLC_SELF) return HLC_E_UNSUPPORTED;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  try {
    return sort_output(
        batch_impl(jobs, njobs, a_ra, a_dec, b_ra, b_dec, out_pairs, out_sep_arcsec, job_pair_count, opts),
        out_pairs, out_sep_arcsec, opts, int64_t(1) << 31, int64_t(1) << 31);
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

}  // extern "C"

namespace hlc {
namespace {

// Resources of one streaming call, released in one place.
// Per-call streams and events; buffers are carved from the device's
// streaming arenas (arena 0: uploads, histogram, ring; arena 1: chunk-ordered
// copies, sized once the halo copies are counted).
struct StreamCall {
  Device* d = nullptr;
  hipStream_t s_copy = nullptr, s_d2h = nullptr;
  hipEvent_t ev_copy = nullptr, ev_done = nullptr, ev_d2h[2] = {nullptr, nullptr};
  hipEvent_t ev_slab[2] = {nullptr, nullptr};  // A slab copied into buffer k
  hipEvent_t ev_free[2] = {nullptr, nullptr};  // buffer k's slab cross-matched
  ~StreamCall() {
    if (s_copy) (void)hipStreamSynchronize(s_copy);
    if (s_d2h) (void)hipStreamSynchronize(s_d2h);
    for (hipEvent_t e : {ev_copy, ev_done, ev_d2h[0], ev_d2h[1], ev_slab[0], ev_slab[1], ev_free[0], ev_free[1]})
      if (e) (void)hipEventDestroy(e);
    if (s_copy) (void)hipStreamDestroy(s_copy);
    if (s_d2h) (void)hipStreamDestroy(s_d2h);
  }
  // grow arena k to hold `bytes` (its previous contents are dropped)
  int reserve(int k, size_t bytes) {
    if (bytes <= d->sarena_bytes[k]) return HLC_OK;
    (void)hipDeviceSynchronize();
    if (d->sarena[k]) (void)hipFree(d->sarena[k]);
    d->sarena[k] = nullptr;
    d->sarena_bytes[k] = 0;
    HLC_CHECK(dev_alloc(&d->sarena[k], bytes));
    d->sarena_bytes[k] = bytes;
    return HLC_OK;
  }
  int reserve_host(size_t bytes) {
    if (bytes <= d->harena_bytes) return HLC_OK;
    if (d->harena) (void)hipHostFree(d->harena);
    d->harena = nullptr;
    d->harena_bytes = 0;
    if (alloc_fails(bytes)) return HLC_E_NOMEM;
    HLC_TRY(hipHostMalloc(&d->harena, bytes, hipHostMallocDefault));
    d->harena_bytes = bytes;
    return HLC_OK;
  }
};

// ---------------------------------------------------------------------------
// eq. (5) transfer model: T(d) = alpha + beta d, fitted to timed copies
// ---------------------------------------------------------------------------
struct TransferModel {
  bool have = false;
  hlc_transfer m{};
};
TransferModel g_tm[MAX_DEVICES];

void fit_line(const std::vector<double>& x, const std::vector<double>& y, double& a, double& b, double& r2) {
  const double n = (double)x.size();
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    sx += x[i];
    sy += y[i];
    sxx += x[i] * x[i];
    sxy += x[i] * y[i];
  }
  b = (n * sxy - sx * sy) / (n * sxx - sx * sx);
  a = (sy - b * sx) / n;
  double my = sy / n, ss_tot = 0, ss_res = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    const double f = a + b * x[i];
    ss_res += (y[i] - f) * (y[i] - f);
    ss_tot += (y[i] - my) * (y[i] - my);
  }
  r2 = ss_tot > 0 ? 1.0 - ss_res / ss_tot : 1.0;
}

int measure_transfer(int dev_id, hlc_transfer* out) {
  TransferModel& T = g_tm[dev_id];
  if (T.have) {
    *out = T.m;
    return HLC_OK;
  }
  const size_t maxb = size_t(1) << 26;
  void *h = nullptr, *d = nullptr;
  if (alloc_fails(maxb)) return HLC_E_NOMEM;
  HLC_TRY(hipHostMalloc(&h, maxb, hipHostMallocDefault));
  if (hipMalloc(&d, maxb) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(h);
    return HLC_E_NOMEM;
  }
  std::memset(h, 1, maxb);
  hipStream_t s;
  hipEvent_t e0, e1;
  int st = HLC_OK;
  if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = HLC_E_DEVICE;
  } else {
    std::vector<double> xs, yh, yd;
    for (int k = 0; k <= 26; k += 2) {
      const size_t bytes = size_t(1) << k;
      for (int dir = 0; dir < 2; ++dir) {
        double best = 1e30;
        for (int rep = 0; rep < 5; ++rep) {  // best of five: transient noise only adds time
          (void)hipEventRecord(e0, s);
          if (dir == 0) (void)hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);
          else (void)hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          best = std::min(best, (double)ms * 1e-3);
        }
        (dir == 0 ? yh : yd).push_back(best);
      }
      xs.push_back((double)bytes);
    }
    fit_line(xs, yh, T.m.alpha_h2d, T.m.beta_h2d, T.m.r2_h2d);
    fit_line(xs, yd, T.m.alpha_d2h, T.m.beta_d2h, T.m.r2_d2h);
    T.have = true;
    *out = T.m;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
  }
  (void)hipFree(d);
  (void)hipHostFree(h);
  return st;
}

// Frame of a streamed call from B's footprint widened by the radius: every
// A source with a partner lies inside it (A sources outside are clamped into
// the edge zones and bins, where they find nothing). The whole RA circle when
// the widened box spans 170 deg or more, crosses RA 0/360 or comes within a
// degree of a pole.
Frame frame_around(const Box& b, double r_arcsec) {
  Frame f;
  if (!b.any) return f;
  const double rr = r_arcsec / 3600.0 * (1.0 + 1e-9) + 1e-9;
  f.dec_lo = std::max(-90.0, b.dlo - rr);
  f.dec_hi = std::min(90.0, b.dhi + rr);
  const double dmax = std::max(std::fabs(f.dec_lo), std::fabs(f.dec_hi));
  if (dmax + rr >= 89.0) return f;
  const double d2r = M_PI / 180.0;
  const double D = std::asin(std::min(1.0, std::sin(rr * d2r) / std::cos(dmax * d2r))) / d2r * (1.0 + 1e-9) + 1e-9;
  const double lo = b.rlo - D, hi = b.rhi + D;
  if (lo < 0.0 || hi > 360.0 || hi - lo >= 170.0) return f;
  f.full_ra = false;
  f.ra_lo = lo;
  f.ra_span = hi - lo;
  return f;
}

// Cross-match of one A slab (device coordinates, m sources) with the
// partitioned B; pairs into (rp, rs) of capacity cap, their count (or the
// required count) in *found.
int slab_match(Device& dev, const double* a_ra, const double* a_dec, uint32_t m, const Side& B,
               uint32_t* zstartB, const Geom& g, double r_arcsec, bool fp32, Caps& caps, hlc_pair* rp,
               double* rs, int64_t cap, int64_t* found, const hlc_opts* o, hipStream_t s) {
  for (int attempt = 0; attempt < 3; ++attempt) {
    Side A;
    SortScratch scA;
    MatchWs w;
    auto lay = [&](Carve& c) {
      carve_side(c, A, m, !fp32, fp32, m, false);
      carve_sort(c, scA, m);
      carve_match_ws(c, w, m, g, caps, false);
    };
    Carve sizing{nullptr};
    lay(sizing);
    HLC_CHECK(ensure_ws(dev, sizing.off + 256));
    Carve c{(char*)dev.ws};
    lay(c);
    w.zstartB = zstartB;
    launch_zero_counters(dev.cnt, s);
    partition_keys(dev, a_ra, a_dec, m, g, false, !fp32, fp32, scA, 1u, A, NO_SLOTS, s);
    HLC_CHECK(partition_sort(dev, g, !fp32, fp32, scA, A, NO_SLOTS, s));
    match(dev, A, B, g, r_arcsec, fp32, false, false, Radii{nullptr, nullptr, 0.0}, w, rp,
          (o->flags & HLC_NO_SEP) ? nullptr : rs, (uint64_t)cap, false, tuned_items(o), s);
    HLC_CHECK(read_counters(dev, s, false));
    const Counters& h = *dev.cnt_host;
    if (h.err) return HLC_E_INVAL;
    if (regrow(dev, h, (uint64_t)cap, caps)) continue;
    *found = (int64_t)h.n_pairs;
    return h.n_pairs > (unsigned long long)cap ? HLC_E_OVERFLOW : HLC_OK;
  }
  return HLC_E_NOMEM;
}

// Streaming form. B is copied once, partitioned once (frame from its
// footprint) and stays resident; A follows in input-order slabs, two device
// buffers deep, each slab's copy overlapping the previous slab's
// cross-match. Each slab's pairs go back through one half of a device ring
// while the other half is being filled. Slabs are sized from the eq. (5)
// transfer model.
int stream_impl(const double* a_ra_h, const double* a_dec_h, int64_t na, const double* b_ra_h,
                const double* b_dec_h, int64_t nb, double r_arcsec, hlc_sink sink, void* user,
                const hlc_opts* o) {
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  hipStream_t s = (hipStream_t)o->stream;
  const bool fp32 = o->precision == HLC_FP32_RECHECK;
  std::memset(&g_stats, 0, sizeof(g_stats));
  g_stats.na = na;
  g_stats.nb = nb;
  *o->n_pairs = 0;
  StreamCall sc;
  sc.d = dev;
  // non-blocking: a caller on the legacy null stream would otherwise
  // serialise the copies with the compute (every dependency is an event)
  HLC_TRY(hipStreamCreateWithFlags(&sc.s_copy, hipStreamNonBlocking));
  HLC_TRY(hipStreamCreateWithFlags(&sc.s_d2h, hipStreamNonBlocking));
  HLC_TRY(hipEventCreateWithFlags(&sc.ev_copy, hipEventDisableTiming));
  HLC_TRY(hipEventCreateWithFlags(&sc.ev_done, hipEventDisableTiming));
  for (auto* e : {&sc.ev_d2h[0], &sc.ev_d2h[1], &sc.ev_slab[0], &sc.ev_slab[1], &sc.ev_free[0], &sc.ev_free[1]})
    HLC_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  for (hipEvent_t e : sc.ev_free) HLC_TRY(hipEventRecord(e, s));  // both A buffers start free

  // A slab size: with per-slab fixed cost s_fix = alpha_h2d + alpha_d2h +
  // launch overhead (about 30 launches and two synchronisations) and
  // whole-job time W (A over the link, about one pair per A source back,
  // compute at ~3e9 sources/s), about sqrt(W / s_fix) slabs balance the
  // fixed costs against the pipeline's fill and drain.
  int dev_id = 0;
  HLC_TRY(hipGetDevice(&dev_id));
  hlc_transfer tm{};
  int64_t SLAB = int64_t(1) << 24;
  if (measure_transfer(dev_id, &tm) == HLC_OK && tm.beta_h2d > 0 && tm.beta_d2h > 0) {
    const double s_fix = std::max(tm.alpha_h2d, 0.0) + std::max(tm.alpha_d2h, 0.0) + 3.0e-4;
    const double W = tm.beta_h2d * 16.0 * (double)na + tm.beta_d2h * 16.0 * (double)na + (double)na / 3.0e9;
    const double k = std::sqrt(W / s_fix);
    SLAB = (int64_t)std::min(std::max((double)na / std::max(k, 1.0), 1048576.0), 33554432.0);
  }
  SLAB = std::max<int64_t>(std::min<int64_t>(SLAB, na), 1);
  const int64_t nslab = (na + SLAB - 1) / SLAB;

  // ring: two halves, each drained to its own pinned host staging area
  const int64_t ring = o->capacity > 0 ? o->capacity : (int64_t(1) << 25);
  const int64_t half = std::max<int64_t>(ring / 2, 1024);
  const uint32_t nB = (uint32_t)nb;
  hlc_pair* d_pairs;
  double* d_sep;
  double *B_ra, *B_dec;
  uint32_t* zstartB;
  Side B;
  SortScratch scB;
  auto lay0 = [&](Carve& c) {
    d_pairs = c.take<hlc_pair>(2 * half);
    d_sep = c.take<double>(2 * half);
    B_ra = c.take<double>(std::max(nB, 1u));
    B_dec = c.take<double>(std::max(nB, 1u));
    carve_side(c, B, 2 * nB, !fp32, fp32, nB);
    carve_sort(c, scB, 2 * nB);
    zstartB = c.take<uint32_t>(65537);
  };
  double* A_ra[2];
  double* A_dec[2];
  auto lay1 = [&](Carve& c) {
    for (int k = 0; k < 2; ++k) {
      A_ra[k] = c.take<double>((size_t)SLAB);
      A_dec[k] = c.take<double>((size_t)SLAB);
    }
  };
  {
    Carve z{nullptr};
    lay0(z);
    HLC_CHECK(sc.reserve(0, z.off + 256));
    Carve c{(char*)dev->sarena[0]};
    lay0(c);
    Carve z1{nullptr};
    lay1(z1);
    HLC_CHECK(sc.reserve(1, z1.off + 256));
    Carve c1{(char*)dev->sarena[1]};
    lay1(c1);
  }
  hlc_pair* h_pairs[2];
  double* h_sep[2];
  {
    HLC_CHECK(sc.reserve_host((size_t)half * 2 * (sizeof(hlc_pair) + sizeof(double)) + 1024));
    char* hp = (char*)dev->harena;
    for (int k = 0; k < 2; ++k) {
      h_pairs[k] = (hlc_pair*)hp;
      hp += (size_t)half * sizeof(hlc_pair);
      h_sep[k] = (double*)hp;
      hp += (size_t)half * sizeof(double);
    }
  }
  auto copy_slab = [&](int64_t k) -> int {
    const int b = (int)(k & 1);
    const int64_t a0 = k * SLAB, m = std::min(SLAB, na - a0);
    // the buffer's previous slab must be done with it
    HLC_TRY(hipStreamWaitEvent(sc.s_copy, sc.ev_free[b], 0));
    HLC_TRY(hipMemcpyAsync(A_ra[b], a_ra_h + a0, (size_t)m * 8, hipMemcpyHostToDevice, sc.s_copy));
    HLC_TRY(hipMemcpyAsync(A_dec[b], a_dec_h + a0, (size_t)m * 8, hipMemcpyHostToDevice, sc.s_copy));
    HLC_TRY(hipEventRecord(sc.ev_slab[b], sc.s_copy));
    return HLC_OK;
  };

  // 1. B, then the first A slab, over the link
  if (nB) {
    HLC_TRY(hipMemcpyAsync(B_ra, b_ra_h, (size_t)nB * 8, hipMemcpyHostToDevice, sc.s_copy));
    HLC_TRY(hipMemcpyAsync(B_dec, b_dec_h, (size_t)nB * 8, hipMemcpyHostToDevice, sc.s_copy));
  }
  HLC_TRY(hipEventRecord(sc.ev_copy, sc.s_copy));
  if (nslab > 0) HLC_CHECK(copy_slab(0));
  HLC_TRY(hipStreamWaitEvent(s, sc.ev_copy, 0));

  // 2. the frame from B's footprint; B partitioned once
  launch_zero_counters(dev->cnt, s);
  launch_extent(B_ra, B_dec, nB, dev->cnt, s);
  HLC_CHECK(read_counters(*dev, s, false));
  const Frame f = frame_around(read_box(*dev->cnt_host), r_arcsec);
  const Geom g = make_geom(r_arcsec, tuned_height(o), na, nb, tuned_bins(o), f);
  launch_zero_counters(dev->cnt, s);
  HLC_CHECK(partition(*dev, B_ra, B_dec, nB, g, true, !fp32, fp32, scB, 2u, B, NO_SLOTS, s));
  launch_zone_starts(B.keys, B.cnt, g, zstartB, s);
  HLC_CHECK(read_counters(*dev, s, false));
  if (dev->cnt_host->err) return HLC_E_INVAL;
  const uint32_t ne = nB + (uint32_t)dev->cnt_host->n_halo;
  B.cnt = DevCount{ne, ne, nullptr};  // final: the counters are reused per slab
  g_stats.nb_halo = ne;
  g_stats.n_zones = g.nz;
  g_stats.ra_bits = g.rb;
  g_stats.zone_height_arcsec = g.h_deg * 3600.0;

  // 3. A slabs through the cross-match; pairs leave through the ring
  int64_t total = 0;
  int64_t pending[2] = {-1, -1};
  int slot = 0;
  auto drain = [&](int h) -> int {
    if (pending[h] < 0) return HLC_OK;
    HLC_TRY(hipEventSynchronize(sc.ev_d2h[h]));
    const int64_t n = pending[h];
    pending[h] = -1;
    if (n > 0 && sink(h_pairs[h], (o->flags & HLC_NO_SEP) ? nullptr : h_sep[h], n, user) != 0)
      return HLC_E_INVAL;
    return HLC_OK;
  };
  Caps caps = initial_caps(*dev, 2 * (uint64_t)SLAB, (uint64_t)half, true);
  for (int64_t k = 0; k < nslab; ++k) {
    const int b = (int)(k & 1);
    const int64_t a0 = k * SLAB, m = std::min(SLAB, na - a0);
    if (k + 1 < nslab) HLC_CHECK(copy_slab(k + 1));
    HLC_TRY(hipStreamWaitEvent(s, sc.ev_slab[b], 0));
    // sub-ranges of the slab: a range with more pairs than half the ring is
    // split in two
    std::vector<std::pair<int64_t, int64_t>> todo{{0, m}};
    while (!todo.empty()) {
      const auto [u0, um] = todo.back();
      todo.pop_back();
      if (um == 0) continue;
      HLC_CHECK(drain(slot));  // this half's previous batch has reached the host
      hlc_pair* rp = d_pairs + slot * half;
      double* rs = d_sep + slot * half;
      int64_t found = 0;
      const int st = slab_match(*dev, A_ra[b] + u0, A_dec[b] + u0, (uint32_t)um, B, zstartB, g, r_arcsec, fp32,
                                caps, rp, rs, half, &found, o, s);
      if (st == HLC_E_OVERFLOW) {
        if (um == 1) return HLC_E_OVERFLOW;  // one source has more pairs than half the ring
        const int64_t h1 = um / 2;
        todo.push_back({u0 + h1, um - h1});
        todo.push_back({u0, h1});
        continue;
      }
      if (st != HLC_OK) return st;
      launch_offset_pairs(reinterpret_cast<uint2*>(rp), (uint32_t)found, (uint32_t)(a0 + u0), s);
      HLC_TRY(hipEventRecord(sc.ev_done, s));
      HLC_TRY(hipStreamWaitEvent(sc.s_d2h, sc.ev_done, 0));
      if (found > 0) {
        HLC_TRY(hipMemcpyAsync(h_pairs[slot], rp, found * sizeof(hlc_pair), hipMemcpyDeviceToHost, sc.s_d2h));
        if (!(o->flags & HLC_NO_SEP))
          HLC_TRY(hipMemcpyAsync(h_sep[slot], rs, found * sizeof(double), hipMemcpyDeviceToHost, sc.s_d2h));
      }
      HLC_TRY(hipEventRecord(sc.ev_d2h[slot], sc.s_d2h));
      pending[slot] = found;
      total += found;
      slot ^= 1;
    }
    HLC_TRY(hipEventRecord(sc.ev_free[b], s));
  }
  HLC_CHECK(drain(slot));
  HLC_CHECK(drain(slot ^ 1));
  g_stats.n_pairs = total;
  *o->n_pairs = total;
  return HLC_OK;
}

}  // namespace
}  // namespace hlc

extern "C" {

int hlc_xmatch_stream(const double* a_ra_host, const double* a_dec_host, int64_t na,
                      const double* b_ra_host, const double* b_dec_host, int64_t nb, double r_arcsec,
                      hlc_sink sink, void* user, const hlc_opts* opts) {
  int st = check_common(r_arcsec, na, nb, opts);
  if (st) return st;
  if (!sink) return HLC_E_INVAL;
  if ((na > 0 && (!a_ra_host || !a_dec_host)) || (nb > 0 && (!b_ra_host || !b_dec_host)))
    return HLC_E_INVAL;
  if (opts->flags & (HLC_SELF | HLC_SORTED)) return HLC_E_UNSUPPORTED;  // pairs arrive per chunk
  try {
    return stream_impl(a_ra_host, a_dec_host, na, b_ra_host, b_dec_host, nb, r_arcsec, sink, user, opts);
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

int hlc_transfer_model(hlc_transfer* out) {
  if (!out) return HLC_E_INVAL;
  try {
    Device* dev = nullptr;
    int dev_id = 0;
    HLC_CHECK(get_device(&dev, &dev_id));
    return measure_transfer(dev_id, out);
  } catch (...) {
    return HLC_E_DEVICE;
  }
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
  for (auto& B : g_bstate) {
    drop_graph(B);
    if (B.tables) (void)hipFree(B.tables);
    if (B.st) (void)hipStreamDestroy(B.st);
    if (B.st2) (void)hipStreamDestroy(B.st2);
    for (hipEvent_t e : {B.ev_in, B.ev_out, B.ev_t0, B.ev_t1, B.ev_fork[0], B.ev_fork[1], B.ev_join[0],
                         B.ev_join[1]})
      if (e) (void)hipEventDestroy(e);
    B = BatchState();
  }
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
