// xmatch_api.hip -- the single-call entry points: hlc_xmatch (and its
// self-match mode), hlc_xmatch_radii (eq. (4) per-source radii) and
// hlc_xmatch_quad (the paper's HEALPix + quad-direction partition, emulated).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "host.hpp"

namespace hlc {
namespace {

int xmatch_impl(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                double* out_sep, const hlc_opts* o, Caps& caps, bool* again, const Radii& rad) {
  *again = false;
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  hipStream_t s = (hipStream_t)o->stream;
  const bool prof = (o->flags & HLC_PROFILE) != 0;
  const int plevel = prof_level(o->flags);
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
  // FP32: B in the sorted certification layout when the last FP32 call on
  // this device had that many candidates per B entry
  const bool sorted_b = fp32 && dev->cand_per_b >= SORTED_RADEC_MIN;
  auto lay = [&](Carve& c) {
    // A is read in place: the filter gathers its records itself
    if (!self) {
      carve_side(c, A, nA, !fp32, fp32, nA, false);
      carve_sort(c, scA, nA);
    }
    carve_side(c, B, 2 * nB, !fp32, fp32, nB, true, sorted_b);
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
      // B's on the caller's stream, launched first (B's chain is the longer
      // one), A's beside it on the side stream, where A's sort follows (the
      // places of B's buffers do not depend on the frame either)
      HLC_TRY(hipEventRecord(dev->fork, s));
      partition_keys(*dev, b_ra, b_dec, nB, g, true, !fp32, fp32, sc, 2u, B, slB, s);
      HLC_TRY(hipStreamWaitEvent(dev->side, dev->fork, 0));
      partition_keys(*dev, a_ra, a_dec, nA, g, false, !fp32, fp32, scA, 1u, A, slA, dev->side);
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
  // (B's keygen launched first: B's chain is the longer one)
  if (!keep) {
    if (!self) HLC_TRY(hipEventRecord(dev->fork, s));
    partition_keys(*dev, b_ra, b_dec, nB, g, true, !fp32, fp32, sc, 2u, B, slB, s);
    if (!self) {
      HLC_TRY(hipStreamWaitEvent(dev->side, dev->fork, 0));
      partition_keys(*dev, a_ra, a_dec, nA, g, false, !fp32, fp32, scA, 1u, A, slA, dev->side);
    }
  }
  if (self) mark(*dev, slA.keygen, s);
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
        (o->flags & HLC_NO_SEP) ? nullptr : out_sep, (uint64_t)o->capacity, plevel, tuned_items(o), s, dev->side);
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
  else if (plevel == PROF_FILTER) g_stats.t_match_ms = elapsed(dev->ev[13], dev->ev[9]);
  if (fp32) dev->cand_per_b = (double)h.n_cand / (double)std::max<unsigned long long>(1, nb + h.n_halo);
  *o->n_pairs = (int64_t)h.n_pairs;
  return h.n_pairs > (unsigned long long)o->capacity ? HLC_E_OVERFLOW : HLC_OK;
}

// xmatch_impl with the work-buffer retry.
int xmatch_core(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                double* out_sep, const hlc_opts* o, const Radii& rad = Radii{nullptr, nullptr, 0.0}) {
  Device* dev = nullptr;
  HLC_CHECK(get_device(&dev));
  Caps caps = initial_caps(*dev, (uint64_t)(na + nb), (uint64_t)o->capacity, true, false);
  for (int attempt = 0; attempt < 3; ++attempt) {
    bool again = false;
    int st = xmatch_impl(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, out_pairs, out_sep, o, caps, &again, rad);
    if (!again) return st;
  }
  return HLC_E_NOMEM;
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
    Caps caps = initial_caps(*dev, (uint64_t)capA + capB, (uint64_t)opts->capacity, true, true);
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
        carve_side(c, A, capA, true, false);
        carve_side(c, B, capB, true, false);
        A.radec = c.take<double2>(capA);  // sorted (ra, dec): pixel tests
        B.radec = c.take<double2>(capB);
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
      ma.valsA = A.vals;
      ma.valsB = B.vals;
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

}  // extern "C"
