// host.hpp -- host-side pieces that the entry points of libhlc share: the
// per-device context and workspace, the partition geometry and frame, the
// thresholds of the decision, and the two phases of a call:
//   partition(): keygen -> radix sort -> working layout of ONE catalogue
//                (section 4.2's first-level partition, on the GPU);
//   match():     B zone tables -> key index -> group ranges -> filter ->
//                candidate certification -> band list -> packing (section 4.3).
// Each form's own host logic lives in its file: xmatch_api.hip (single
// calls), part_api.hip (reusable partitions), batch_api.hip + tune_cache.hip
// (batched form), stream_api.hip (pinned host catalogues).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/hlc.h"
#include "hlc_kernels.hpp"

namespace hlc {

constexpr int MAX_DEVICES = 64;
constexpr double U64 = 1.1102230246251565e-16;
constexpr double ETA64 = 4e-15;  // bound on |chord_fp64 - chord| (unit sphere)

// ---------------------------------------------------------------------------
// per-device context (context.hip)
// ---------------------------------------------------------------------------
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
  // streaming form: A sources cross-matched per second by the last
  // streaming call's slabs (0: not measured yet)
  double stream_rate = 0.0;
  // A's partition runs on `side` beside B's on the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr;
  // B sorted (the ranges start) and ranges done (the filter may start)
  hipEvent_t bsorted = nullptr, prepped = nullptr;
  // staging sizes that earlier calls needed (grow-only), so a repeated
  // workload does not pay the overflow re-run again
  uint64_t hint_stage = 0, hint_cand = 0;
  // FP32 candidates per B entry of the last FP32 single call: at
  // SORTED_RADEC_MIN or more the next one uses the sorted certification
  // layout for B (see carve_side)
  double cand_per_b = 0.0;
  int ncu = 0;  // compute units (persistent grids)
  bool last_full = true;  // the last call's frame was the whole sphere
  // the footprint sample's result, written by the kernel into mapped host
  // memory (4 values, then the call's sequence number) and polled
  unsigned long long* fmsg_host = nullptr;
  unsigned long long* fmsg_dev = nullptr;
  unsigned long long fseq = 0;
};

extern Device g_dev[MAX_DEVICES];
// statistics of the last call made on the calling thread
extern thread_local hlc_stats g_stats;

inline int map_err(hipError_t e) {
  if (e == hipSuccess) return HLC_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return HLC_E_NOMEM;
  return HLC_E_DEVICE;
}

#define HLC_TRY(x)                            \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return map_err(e_); \
  } while (0)

#define HLC_CHECK(x)             \
  do {                           \
    int s_ = (x);                \
    if (s_ != HLC_OK) return s_; \
  } while (0)

int get_device(Device** out, int* dev_id = nullptr);
// HLC_TEST_FAIL_ALLOC=<bytes>: allocations of at least that size fail
// (failure-injection tests)
bool alloc_fails(size_t bytes);
int dev_alloc(void** p, size_t bytes);
int ensure_ws(Device& d, size_t bytes);
int read_counters(Device& dev, hipStream_t s, bool prof);
float elapsed(hipEvent_t a, hipEvent_t b);
void fill_stats(const Counters& h, int64_t na, int64_t nb, int64_t nbh, const Geom& g);
void fill_times(Device& dev, bool with_partition);
// releases the batched form's per-device state (batch_api.hip)
void batch_release_all();

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

// ---------------------------------------------------------------------------
// geometry, frame and thresholds (geometry.hip)
// ---------------------------------------------------------------------------
inline int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

inline int zone_bits(int64_t nz) { return std::max(1, ceil_log2((uint64_t)nz)); }

inline void set_radius(Geom& g, double r_arcsec) {
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

// Partition geometry: zone height h_as (arcsec; <= 0 = automatic from the
// data density), radius r (halo and windows), frame f.
Geom make_geom(double r_arcsec, double h_as, int64_t na, int64_t nb, int ra_bits, const Frame& f = Frame{});

inline double ext_value(unsigned long long code) {
  double v;
  std::memcpy(&v, &code, 8);
  return v;
}

// Bounding box of the valid sources from the footprint codes (any: at least
// one valid source).
struct Box {
  bool any;
  double dlo, dhi, rlo, rhi;
};
inline Box read_box(const Counters& h) {
  Box b;
  b.any = h.ext[1] != 0ull;
  b.dlo = ext_value(~h.ext[0]) - 90.0;
  b.dhi = ext_value(h.ext[1]) - 90.0;
  b.rlo = ext_value(~h.ext[2]);
  b.rhi = ext_value(h.ext[3]);
  return b;
}

// The frame of a call's data: a sample of both catalogues first; where its
// box covers over a quarter of the sphere the whole sphere is the frame,
// otherwise one pass over every source gives the exact box.
unsigned long long frame_sample(Device& dev, const double* a_ra, const double* a_dec, int64_t na,
                                const double* b_ra, const double* b_dec, int64_t nb, hipStream_t s);
int frame_finish(Device& dev, unsigned long long seq, const double* a_ra, const double* a_dec, int64_t na,
                 const double* b_ra, const double* b_dec, int64_t nb, hipStream_t s, Frame* out);
// the box covers over a quarter of the sphere (the whole sphere is the frame)
bool quarter_sky(const Box& b);
// the frame of an exact box of every valid source (a small margin added)
Frame frame_of_box(const Box& b);
inline bool is_full(const Frame& f) { return f.full_ra && f.dec_lo == -90.0 && f.dec_hi == 90.0; }

inline int key_bits(const Geom& g) { return zone_bits(g.nz) + g.rb + g.fb; }

struct Thresholds {
  double c_r, t_lo64, t_hi64, H_lo, H_hi;
  float c_r32;  // c_r rounded up to FP32
};
Thresholds thresholds(double r_arcsec);

inline int check_opts(const hlc_opts* o) {
  if (!o || !o->n_pairs) return HLC_E_INVAL;
  if (o->capacity < 0) return HLC_E_INVAL;
  if (o->precision != HLC_FP32_RECHECK && o->precision != HLC_FP64) return HLC_E_INVAL;
  if (o->tuning && (o->tuning->ra_bins_log2 < 0 || o->tuning->ra_bins_log2 > 30)) return HLC_E_INVAL;
  return HLC_OK;
}

// Largest catalogue: B's entries (sources plus halo copies, up to twice the
// sources) and every grid rounded up to whole tiles stay below 2^32.
constexpr int64_t MAX_SOURCES = (int64_t(1) << 31) - (int64_t(1) << 16);

inline int check_common(double r_arcsec, int64_t na, int64_t nb, const hlc_opts* o) {
  HLC_CHECK(check_opts(o));
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return HLC_E_INVAL;
  if (na < 0 || nb < 0 || na > MAX_SOURCES || nb > MAX_SOURCES) return HLC_E_INVAL;
  return HLC_OK;
}

inline double tuned_height(const hlc_opts* o) {
  return (o->tuning && o->tuning->zone_height_arcsec > 0) ? o->tuning->zone_height_arcsec : 0.0;
}
inline int tuned_bins(const hlc_opts* o) { return o->tuning ? o->tuning->ra_bins_log2 : 0; }
inline bool tuned_fraction_sort(const hlc_opts* o) { return o->tuning && o->tuning->fraction_sort == 1; }
// lowest key bit the radix sort orders: 0 when the sub-bin bits are sorted too
inline int sort_lo(const Geom& g) { return g.frac_sorted ? 0 : g.fb; }
inline int tuned_items(const hlc_opts* o) {
  return (o->tuning && o->tuning->filter_items > 0) ? o->tuning->filter_items : 1;
}

// ---------------------------------------------------------------------------
// the two phases of a call (pipeline.hip)
// ---------------------------------------------------------------------------
// One partitioned catalogue.
struct Side {
  uint32_t n_src = 0, n_cap = 0;  // sources; entry capacity (2 n_src with a halo)
  DevCount cnt{0, 0, nullptr};    // entries, halo copies included (device-side)
  uint32_t *keys = nullptr, *vals = nullptr;
  Rec64* r64 = nullptr;
  CellRec32* r32 = nullptr;
  // sorted (ra, dec): FP32 form in the sorted certification layout (see
  // carve_side), and the paper-scheme emulation's pixel tests
  double2* radec = nullptr;
  // (ra, dec) of each source, 16 B, written by the keygen in input order
  // (nullptr: the layout reads the caller's coordinates): the sorted records
  // of a gathered side are computed from it, the filter reads a side in
  // place from it, and the certification reads B's positions from it
  double2* srcrad = nullptr;
  const double *ra = nullptr, *dec = nullptr;  // original coordinates (for the band list)
};

// Profiling event slots (HLC_PROFILE): per partition, {after keygen,
// before sort, after sort, after layout}; -1 = not recorded.
struct Slots {
  int keygen, sort_begin, sort, layout;
};
constexpr Slots NO_SLOTS{-1, -1, -1, -1};

inline void mark(Device& dev, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(dev.ev[slot], s);
}

// Partition of one side in two steps (the keygen can run on another stream
// than the sort): keys (and the per-source records) first, then the sort and
// the sorted layout. l64 / l32: the side's records are FP64 / FP32; without
// a sorted layout (sd.r64 / sd.r32 null) the per-source records stay in
// input order and the kernels read them through vals. sorted_ev (optional)
// is recorded once the keys are sorted, before the records are gathered.
void partition_keys(Device& dev, const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
                    bool l64, bool l32, const SortScratch& sc, uint32_t err_bit, Side& sd, const Slots& sl,
                    hipStream_t s);
int partition_sort(Device& dev, const Geom& g, bool l64, bool l32, const SortScratch& sc, Side& sd,
                   const Slots& sl, hipStream_t s, hipEvent_t sorted_ev = nullptr);
int partition(Device& dev, const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
              bool l64, bool l32, const SortScratch& sc, uint32_t err_bit, Side& sd, const Slots& sl,
              hipStream_t s, hipEvent_t sorted_ev = nullptr);

// Coarse index of B's sorted keys: one entry per 2^shift keys, at most 2^18
// (never finer than the sorted key bits: the low fb bits of a sorted key
// array are in input order within a bin, so the index is exact only on
// multiples of 2^fb)
// Below about two FP32 candidates per B entry, reading each candidate's B
// (ra, dec) at random from a 16-B array in input order costs less than
// gathering every entry's into sorted order (measured at 10M x 10M,
// 0.4 per entry: 10 us slower with the gather; at 20M x 20M, 8.7 per entry:
// 0.35-0.5 ms faster).
constexpr double SORTED_RADEC_MIN = 2.0;

struct KeyIndex {
  int shift;
  uint32_t T;
};
inline KeyIndex key_index_dims(const Geom& g) {
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

// pair_regions: pairs staged in regions and compacted (else written straight
// into the caller's buffer by the certification: no pair slots)
Caps initial_caps(const Device& d, uint64_t entries, uint64_t cap, bool stage_cand, bool pair_regions);
void carve_regions(Carve& c, Regions& r, const Caps& k, bool sep);
// True when the call must run again: its band list overflowed, a candidate
// region overflowed, or a pair region overflowed although the caller's
// buffer holds every pair.
bool regrow(Device& d, const Counters& h, uint64_t cap, Caps& k);
OutArgs out_args(hlc_pair* pairs, double* sep, uint64_t cap, uint2* band, uint64_t band_cap,
                 const Regions& reg, Counters* cnt);
// Everything after the partition: ranges, match, certification. With ps the
// ranges run there (ordered by the caller after both sorts), beside B's
// gather on s, and the filter and what follows end on ps. prof: 0 no
// events, PROF_FILTER the filter's two events, PROF_ALL every stage's.
constexpr int PROF_FILTER = 1, PROF_ALL = 2;
void match(Device& dev, const Side& A, const Side& B, const Geom& g, double r_arcsec, bool fp32,
           bool skip_halo_a, bool self_only, const Radii& rad, const MatchWs& w, hlc_pair* out_pairs,
           double* out_sep, uint64_t cap, int prof, int filter_items, hipStream_t s, hipStream_t ps = nullptr);
// the profiling level of a call's flags
inline int prof_level(uint32_t flags) {
  return (flags & HLC_PROFILE) ? PROF_ALL : ((flags & HLC_TIME_FILTER) ? PROF_FILTER : 0);
}
size_t carve_match_ws(Carve& c, MatchWs& w, uint32_t na_entries, const Geom& g, const Caps& caps,
                      bool need_zstart);
// cap entries; n_src > 0 also carves the per-source records of the keygen;
// without `layout` no sorted records are carved (the side is read in place).
// FP32, gathered: with sorted_radec the sorted certification layout (32-B
// per-source records, gathered into sorted cell records and sorted (ra, dec):
// the certification reads a candidate's B (ra, dec) at its sorted position),
// else 16-B cell records and (ra, dec) in separate input-order arrays (the
// gather and the certification then read at random from arrays half the
// size).
void carve_side(Carve& c, Side& sd, uint32_t cap, bool l64, bool l32, uint32_t n_src = 0, bool layout = true,
                bool sorted_radec = false);
void carve_sort(Carve& c, SortScratch& sc, uint32_t nmax);

// the coordinates checked (no pairs: one side is empty)
int validate_only(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                  const double* b_dec, int64_t nb, double r_arcsec, const hlc_opts* o);
inline int bits_for(int64_t n) { return std::max(1, ceil_log2((uint64_t)std::max<int64_t>(n, 2))); }
// HLC_SORTED: the call's pairs, already in the caller's buffers, ordered by
// (a, b) (indices below na and nb).
int sort_output(int st, hlc_pair* pairs, double* sep, const hlc_opts* o, int64_t na, int64_t nb);

}  // namespace hlc
