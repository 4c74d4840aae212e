// part_api.hip -- reusable partitions: hlc_partition builds one catalogue's
// sorted entries and zone starts once; hlc_xmatch_part matches two of them.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "host.hpp"

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
      // FP32: sorted (ra, dec) kept with the part for the certification (its
      // per-source records are scratch)
      carve_side(c, p->side, cap, true, true, 0, true, true);
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
      p->side.srcrad = c.take<double2>(std::max(nn, 1u));
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
    p->side.srcrad = nullptr;
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
    Caps caps = initial_caps(*dev, (uint64_t)A->side.cnt.cap + B->side.cnt.cap, (uint64_t)opts->capacity, true,
                             false);
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
            (opts->flags & HLC_NO_SEP) ? nullptr : out_sep_arcsec, (uint64_t)opts->capacity, prof_level(opts->flags),
            tuned_items(opts), s);
      HLC_CHECK(read_counters(*dev, s, prof));
      const Counters& h = *dev->cnt_host;
      if (regrow(*dev, h, (uint64_t)opts->capacity, caps)) continue;
      fill_stats(h, A->side.n_src, B->side.n_src, B->side.cnt.cap, g);
      if (prof) fill_times(*dev, false);
      else if (prof_level(opts->flags) == PROF_FILTER) g_stats.t_match_ms = elapsed(dev->ev[13], dev->ev[9]);
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
