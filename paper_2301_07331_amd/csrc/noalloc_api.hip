// noalloc_api.hip -- hlc_xmatch_noalloc: the single cross-match call for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc). It runs the same kernels as
// hlc_xmatch, all on the caller's stream, with the call's workspace and its
// device counters carved from `scratch`, a fixed array of this library in
// device memory, and the counters read back into a host array of this file.
// It calls no hipMalloc, hipFree, hipHostMalloc or any other allocating
// routine, and creates no streams or events.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "host.hpp"

namespace hlc {
namespace {

constexpr size_t SCRATCH_BYTES = size_t(128) << 20;  // 128 MiB per device

// The scratch array. In host code its name is only a host-side stand-in:
// kernels and copies are given the device address that hipGetSymbolAddress
// returns for the current device (kept per device below), never `scratch`.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct ScratchDev {
  bool init = false;
  unsigned char* base = nullptr;  // device address of `scratch` on this device
  Counters host_cnt;              // host copy of the counters (plain memory)
  uint64_t hint_stage = 0, hint_cand = 0;
};
ScratchDev g_scratch[MAX_DEVICES];

// Once per device, with that device current: the device address of its copy
// of `scratch`.
int scratch_setup(ScratchDev** out) {
  int dev = 0;
  HLC_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return HLC_E_DEVICE;
  ScratchDev& d = g_scratch[dev];
  if (!d.init) {
    void* p = nullptr;
    HLC_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HLC_E_DEVICE;
    d.base = static_cast<unsigned char*>(p);
    d.init = true;
  }
  *out = &d;
  return HLC_OK;
}

// A call context whose counters and workspace lie in the scratch array: the
// counters in its first 256 bytes, the workspace after them.
Device scratch_context(ScratchDev& d) {
  Device c;
  c.init = true;
  c.cnt = reinterpret_cast<Counters*>(d.base);
  c.cnt_host = &d.host_cnt;
  c.ws = d.base + 256;
  c.ws_bytes = SCRATCH_BYTES - 256;
  c.hint_stage = d.hint_stage;
  c.hint_cand = d.hint_cand;
  return c;
}
static_assert(sizeof(Counters) <= 256, "counters must fit before the workspace");

// Staging estimates sized for calls that fit the scratch (the regular
// call's floors of 4096 slots per region would take most of it); a call
// that exceeds them runs again with the counted sizes, as hlc_xmatch does.
// Pairs go straight into the caller's buffer: no pair slots.
Caps scratch_caps(const ScratchDev& d, uint64_t entries, uint64_t cap) {
  (void)cap;
  Caps k;
  k.band = 1024 + entries / 64;
  k.stage = 0;
  k.cand = std::max<uint64_t>(entries / (2 * NREG) + 64, d.hint_cand);
  return k;
}

int noalloc_impl(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra, const double* b_dec,
                 int64_t nb, double r_arcsec, hlc_pair* out_pairs, double* out_sep, const hlc_opts* o) {
  ScratchDev* sd = nullptr;
  HLC_CHECK(scratch_setup(&sd));
  Device ctx = scratch_context(*sd);
  hipStream_t s = (hipStream_t)o->stream;
  const bool fp32 = o->precision == HLC_FP32_RECHECK;
  if (na == 0 || nb == 0) {
    // nothing can match; the coordinates are still checked
    const size_t n = (size_t)std::max(na, nb);
    if (8 * n + 1024 > ctx.ws_bytes) return HLC_E_UNSUPPORTED;
    const Geom g = make_geom(r_arcsec, 0.0, na, nb, 0);
    uint32_t* k = static_cast<uint32_t*>(ctx.ws);
    uint32_t* v = k + std::max<size_t>(n, 1);
    launch_zero_counters(ctx.cnt, s);
    if (na) launch_keygen(a_ra, a_dec, (uint32_t)na, g, false, 1u, k, v, ctx.cnt, s);
    if (nb) launch_keygen(b_ra, b_dec, (uint32_t)nb, g, false, 2u, k, v, ctx.cnt, s);
    HLC_CHECK(read_counters(ctx, s, false));
    *o->n_pairs = 0;
    std::memset(&g_stats, 0, sizeof(g_stats));
    g_stats.na = na;
    g_stats.nb = nb;
    return ctx.cnt_host->err ? HLC_E_INVAL : HLC_OK;
  }
  // the frame: the exact box of every source (the whole sphere when it
  // covers over a quarter of it)
  launch_zero_counters(ctx.cnt, s);
  launch_extent(a_ra, a_dec, (uint32_t)na, ctx.cnt, s);
  launch_extent(b_ra, b_dec, (uint32_t)nb, ctx.cnt, s);
  HLC_CHECK(read_counters(ctx, s, false));
  const Box box = read_box(*ctx.cnt_host);
  const Frame f = (!box.any || quarter_sky(box)) ? Frame{} : frame_of_box(box);
  Geom g = make_geom(r_arcsec, tuned_height(o), na, nb, tuned_bins(o), f);
  g.frac_sorted = tuned_fraction_sort(o) ? 1 : 0;
  const uint32_t nA = (uint32_t)na, nB = (uint32_t)nb;
  Caps caps = scratch_caps(*sd, (uint64_t)(na + nb), (uint64_t)o->capacity);
  double* sep = (o->flags & HLC_NO_SEP) ? nullptr : out_sep;
  for (int attempt = 0; attempt < 3; ++attempt) {
    Side A, B;
    SortScratch scA, scB;
    MatchWs w;
    auto lay = [&](Carve& c) {
      carve_side(c, A, nA, !fp32, fp32, nA, false);  // A is read in place
      carve_sort(c, scA, nA);
      carve_side(c, B, 2 * nB, !fp32, fp32, nB);
      carve_sort(c, scB, 2 * nB);
      carve_match_ws(c, w, nA, g, caps, true);
    };
    Carve sizing{nullptr};
    lay(sizing);
    if (sizing.off + 256 > ctx.ws_bytes) return HLC_E_UNSUPPORTED;  // beyond the scratch array
    Carve c{static_cast<char*>(ctx.ws)};
    lay(c);
    launch_zero_counters(ctx.cnt, s);
    partition_keys(ctx, a_ra, a_dec, nA, g, false, !fp32, fp32, scA, 1u, A, NO_SLOTS, s);
    partition_keys(ctx, b_ra, b_dec, nB, g, true, !fp32, fp32, scB, 2u, B, NO_SLOTS, s);
    HLC_CHECK(partition_sort(ctx, g, !fp32, fp32, scA, A, NO_SLOTS, s));
    HLC_CHECK(partition_sort(ctx, g, !fp32, fp32, scB, B, NO_SLOTS, s));
    match(ctx, A, B, g, r_arcsec, fp32, false, false, Radii{nullptr, nullptr, 0.0}, w, out_pairs, sep,
          (uint64_t)o->capacity, false, tuned_items(o), s);
    HLC_CHECK(read_counters(ctx, s, false));
    const Counters& h = *ctx.cnt_host;
    if (h.err) {
      *o->n_pairs = 0;
      return HLC_E_INVAL;
    }
    const bool again = regrow(ctx, h, (uint64_t)o->capacity, caps);
    sd->hint_stage = ctx.hint_stage;
    sd->hint_cand = ctx.hint_cand;
    if (again) continue;
    fill_stats(h, na, nb, nb + (int64_t)h.n_halo, g);
    *o->n_pairs = (int64_t)h.n_pairs;
    return h.n_pairs > (unsigned long long)o->capacity ? HLC_E_OVERFLOW : HLC_OK;
  }
  return HLC_E_UNSUPPORTED;
}

}  // namespace
}  // namespace hlc

using namespace hlc;

extern "C" {

int hlc_xmatch_noalloc(const double* a_ra, const double* a_dec, int64_t na, const double* b_ra,
                       const double* b_dec, int64_t nb, double r_arcsec, hlc_pair* out_pairs,
                       double* out_sep_arcsec, const hlc_opts* opts) {
  int st = check_common(r_arcsec, na, nb, opts);
  if (st) return st;
  if ((na > 0 && (!a_ra || !a_dec)) || (nb > 0 && (!b_ra || !b_dec))) return HLC_E_INVAL;
  if (opts->capacity > 0 && (!out_pairs || (!(opts->flags & HLC_NO_SEP) && !out_sep_arcsec)))
    return HLC_E_INVAL;
  if (opts->flags & (HLC_SELF | HLC_SORTED | HLC_PROFILE | HLC_TIME_FILTER)) return HLC_E_UNSUPPORTED;
  try {
    return noalloc_impl(a_ra, a_dec, na, b_ra, b_dec, nb, r_arcsec, out_pairs, out_sep_arcsec, opts);
  } catch (const std::bad_alloc&) {
    return HLC_E_NOMEM;
  } catch (...) {
    return HLC_E_DEVICE;
  }
}

}  // extern "C"
