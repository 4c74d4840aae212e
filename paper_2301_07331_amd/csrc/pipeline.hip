// pipeline.hip -- the two phases that every cross-match entry point runs:
// the partition of one catalogue (keygen, radix sort, working layout) and
// the match (ranges, filter, certification, packing), plus workspace carving
// and the optional (a, b) ordering of the output.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "host.hpp"

namespace hlc {

// Source i's value is i: the keygen leaves it to the sort's first pass when
// a pass runs (the entries' capacity above one, sorted key bits present).
static bool iota_values(const Geom& g, const Side& sd) {
  return sd.n_cap > 1 && radix_passes(key_bits(g), sort_lo(g)) > 0;
}

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
  sd.n_cap = halo ? 2 * n : n;
  // the keygen also counts the first radix pass's digits of the tiles it alone fills
  const KeygenHist kh{sc.counts, sd.n_cap, sort_lo(g)};
  launch_keygen(ra, dec, n, g, halo, err_bit, kk, vv, dev.cnt, s, sd.srcrad, &kh, iota_values(g, sd));
  mark(dev, sl.keygen, s);
  sd.cnt = halo ? DevCount{n, 2 * n, &dev.cnt->n_halo} : DevCount{n, n, nullptr};
}

int partition_sort(Device& dev, const Geom& g, bool l64, bool l32, const SortScratch& sc, Side& sd,
                   const Slots& sl, hipStream_t s, hipEvent_t sorted_ev) {
  const int bits = key_bits(g);
  const bool from_alt = (radix_passes(bits, sort_lo(g)) & 1) != 0;
  mark(dev, sl.sort_begin, s);
  radix_sort(sd.keys, sd.vals, sd.cnt, bits, sc, s, from_alt, sort_lo(g), keygen_hist_tiles(sd.n_src),
             iota_values(g, sd) ? sd.n_src : 0u);
  mark(dev, sl.sort, s);
  if (sorted_ev) HLC_TRY(hipEventRecord(sorted_ev, s));
  // the sorted records from the keygen's (ra, dec) records when it wrote
  // them (one random line per entry), else from the caller's arrays
  if (l64 && sd.r64) launch_layout64(sd.vals, sd.cnt, sd.ra, sd.dec, sd.r64, s, sd.srcrad);
  if (l32 && sd.r32) launch_layout32(sd.vals, sd.cnt, sd.ra, sd.dec, sd.r32, sd.radec, s, sd.srcrad);
  mark(dev, sl.layout, s);
  return HLC_OK;
}

int partition(Device& dev, const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
              bool l64, bool l32, const SortScratch& sc, uint32_t err_bit, Side& sd,
              const Slots& sl, hipStream_t s, hipEvent_t sorted_ev) {
  partition_keys(dev, ra, dec, n, g, halo, l64, l32, sc, err_bit, sd, sl, s);
  return partition_sort(dev, g, l64, l32, sc, sd, sl, s, sorted_ev);
}

uint64_t stage_guess(uint64_t cap) {
  const uint64_t s = cap / NREG + cap / (4 * NREG) + 4096;
  return std::min<uint64_t>(s, 1ull << 22);
}

Caps initial_caps(const Device& d, uint64_t entries, uint64_t cap, bool stage_cand, bool pair_regions) {
  Caps k;
  k.band = (1u << 20) + entries / 64;
  k.stage = pair_regions ? std::max(stage_guess(cap), d.hint_stage) : 0;
  k.cand = stage_cand ? std::max(std::min<uint64_t>(entries / (2 * NREG) + 4096, 1ull << 22), d.hint_cand) : 0;
  return k;
}

void carve_regions(Carve& c, Regions& r, const Caps& k, bool sep) {
  r.fill = c.take<unsigned long long>((size_t)NREG * REG_STRIDE);
  r.cfill = c.take<unsigned long long>((size_t)NREG * REG_STRIDE);
  r.S = k.stage;
  r.pairs = k.stage ? c.take<uint2>((size_t)NREG * k.stage) : nullptr;
  r.sep = (sep && k.stage) ? c.take<double>((size_t)NREG * k.stage) : nullptr;
  r.Sc = k.cand;
  r.cand = k.cand ? c.take<Cand>((size_t)NREG * k.cand) : nullptr;
  r.cpre = c.take<unsigned long long>((size_t)NREG + 1);
}

// True when the call must run again: its band list overflowed, a candidate
// region overflowed, or a pair region (if pairs are staged) overflowed
// although the caller's buffer holds every pair.
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
  if (!again && k.stage && h.n_pairs <= cap && h.region_max > k.stage) {
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
           hlc_pair* out_pairs, double* out_sep, uint64_t cap, int prof, int filter_items, hipStream_t s,
           hipStream_t ps) {
  // zone tables, key index and ranges need only the sorted keys: on ps
  // (ordered by the caller after both sorts) they overlap B's gather on s
  if (!ps) ps = s;
  Thresholds th = thresholds(r_arcsec);
  const KeyIndex ki = key_index_dims(g);
  launch_key_index(B.keys, B.cnt, ki.shift, ki.T, w.kidx, ps);
  const uint32_t* zstart = w.zstartB;
  // zone starts from the index when zone boundaries fall on its entries (with
  // the zone tables in the same launch), else searched
  const bool from_index = !zstart && g.rb + g.fb >= ki.shift;
  if (from_index) {
    launch_zone_starts_index(w.kidx, ki.shift, ki.T, B.cnt, g, w.zstart_buf, ps, w.zmarg, w.zdelta);
  } else {
    launch_zone_tables(g, w.zmarg, w.zdelta, ps);
    if (!zstart) launch_zone_starts(B.keys, B.cnt, g, w.zstart_buf, ps);
  }
  if (!zstart) zstart = w.zstart_buf;
  launch_ranges(A.keys, A.cnt, w.kidx, ki.shift, ki.T, B.keys, zstart, w.zmarg, w.zdelta, g, w.ranges, ps);
  if (prof >= PROF_ALL) (void)hipEventRecord(dev.ev[8], ps);
  // the candidate regions are cleared before the join, beside the ranges
  // certified pairs go straight into the caller's buffer (no pair regions)
  OutArgs oa = out_args(out_pairs, out_sep, cap, w.band, w.band_cap, w.reg, dev.cnt);
  oa.direct = 1;
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
  ma.srcradA = A.srcrad;
  ma.srcradB = B.srcrad;
  ma.radecA = A.radec;
  ma.radecB = B.radec;
  ma.keysA = A.keys;
  ma.keysB = B.keys;
  ma.c_r32 = th.c_r32;
  ma.valsA = A.vals;
  ma.valsB = B.vals;
  if (!(fp32 ? (const void*)A.r32 : (const void*)A.r64)) {
    ma.a_in_place = 1;
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
  if (prof >= PROF_ALL) (void)hipEventRecord(dev.ev[10], ts);
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
void carve_side(Carve& c, Side& sd, uint32_t cap, bool l64, bool l32, uint32_t n_src, bool layout,
                bool sorted_radec) {
  cap = std::max(cap, 1u);
  sd.keys = c.take<uint32_t>(cap);
  sd.vals = c.take<uint32_t>(cap);
  sd.r64 = (l64 && layout) ? c.take<Rec64>(cap) : nullptr;
  sd.r32 = (l32 && layout) ? c.take<CellRec32>(cap) : nullptr;
  const bool sorted = l32 && layout && sorted_radec;
  sd.radec = sorted ? c.take<double2>(cap) : nullptr;
  // the one per-source record: (ra, dec), 16 B, written by the keygen; the
  // layout computes a gathered side's sorted records from it, the filter a
  // side read in place, and the certification reads it for B's positions
  // (unless they are sorted too)
  sd.srcrad = ((l64 || l32) && n_src) ? c.take<double2>(n_src) : nullptr;
}

void carve_sort(Carve& c, SortScratch& sc, uint32_t nmax) {
  nmax = std::max(nmax, 1u);
  sc.keys_alt = c.take<uint32_t>(nmax);
  sc.vals_alt = c.take<uint32_t>(nmax);
  sc.counts = c.take<uint32_t>(sort_counts_len(nmax));
  sc.digit_totals = c.take<uint32_t>(sort_digit_totals_len(nmax));
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

}  // namespace hlc
