// stream_api.hip -- catalogues in pinned host memory: the eq. (5) transfer
// model and the streaming form (resident B, A slabs on copy streams, pairs
// through a device ring to a host sink).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "host.hpp"

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
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;    // compute-rate timing
  ~StreamCall() {
    if (s_copy) (void)hipStreamSynchronize(s_copy);
    if (s_d2h) (void)hipStreamSynchronize(s_d2h);
    for (hipEvent_t e : {ev_copy, ev_done, ev_d2h[0], ev_d2h[1], ev_slab[0], ev_slab[1], ev_free[0], ev_free[1],
                         ev_t0, ev_t1})
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
  HLC_TRY(hipEventCreate(&sc.ev_t0));
  HLC_TRY(hipEventCreate(&sc.ev_t1));

  // A slab size: with per-slab fixed cost s_fix = alpha_h2d + alpha_d2h +
  // launch overhead (about 30 launches and two synchronisations) and
  // whole-job time W (A over the link, about one pair per A source back,
  // and the cross-match at the device's measured rate), about
  // sqrt(W / s_fix) slabs balance the fixed costs against the pipeline's
  // fill and drain. The rate is the one the previous streaming call on this
  // device measured over its slabs; the first call measures B's partition
  // instead (A sources cost about as much as B's, plus the filter).
  int dev_id = 0;
  HLC_TRY(hipGetDevice(&dev_id));
  hlc_transfer tm{};
  const bool have_tm = measure_transfer(dev_id, &tm) == HLC_OK && tm.beta_h2d > 0 && tm.beta_d2h > 0;
  int64_t SLAB = 0, nslab = 0;
  auto choose_slab = [&](double rate) {
    SLAB = int64_t(1) << 24;
    if (have_tm && rate > 0) {
      const double s_fix = std::max(tm.alpha_h2d, 0.0) + std::max(tm.alpha_d2h, 0.0) + 3.0e-4;
      const double W = tm.beta_h2d * 16.0 * (double)na + tm.beta_d2h * 16.0 * (double)na + (double)na / rate;
      const double k = std::sqrt(W / s_fix);
      SLAB = (int64_t)std::min(std::max((double)na / std::max(k, 1.0), 1048576.0), 33554432.0);
    }
    SLAB = std::max<int64_t>(std::min<int64_t>(SLAB, na), 1);
    nslab = (na + SLAB - 1) / SLAB;
  };
  const bool rate_known = dev->stream_rate > 0;
  if (rate_known) choose_slab(dev->stream_rate);

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
  }
  auto carve_slabs = [&]() -> int {
    Carve z1{nullptr};
    lay1(z1);
    HLC_CHECK(sc.reserve(1, z1.off + 256));
    Carve c1{(char*)dev->sarena[1]};
    lay1(c1);
    return HLC_OK;
  };
  if (rate_known) HLC_CHECK(carve_slabs());
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
  if (rate_known && nslab > 0) HLC_CHECK(copy_slab(0));
  HLC_TRY(hipStreamWaitEvent(s, sc.ev_copy, 0));

  // 2. the frame from B's footprint; B partitioned once
  launch_zero_counters(dev->cnt, s);
  launch_extent(B_ra, B_dec, nB, dev->cnt, s);
  HLC_CHECK(read_counters(*dev, s, false));
  const Frame f = frame_around(read_box(*dev->cnt_host), r_arcsec);
  const Geom g = make_geom(r_arcsec, tuned_height(o), na, nb, tuned_bins(o), f);
  launch_zero_counters(dev->cnt, s);
  HLC_TRY(hipEventRecord(sc.ev_t0, s));
  HLC_CHECK(partition(*dev, B_ra, B_dec, nB, g, true, !fp32, fp32, scB, 2u, B, NO_SLOTS, s));
  launch_zone_starts(B.keys, B.cnt, g, zstartB, s);
  HLC_TRY(hipEventRecord(sc.ev_t1, s));
  HLC_CHECK(read_counters(*dev, s, false));
  if (dev->cnt_host->err) return HLC_E_INVAL;
  if (!rate_known) {
    const double t = (double)elapsed(sc.ev_t0, sc.ev_t1) * 1e-3;
    choose_slab(t > 0 ? (double)std::max(nB, 1u) / t : 0.0);
    HLC_CHECK(carve_slabs());
    if (nslab > 0) HLC_CHECK(copy_slab(0));
  }
  const uint32_t ne = nB + (uint32_t)dev->cnt_host->n_halo;
  B.cnt = DevCount{ne, ne, nullptr};  // final: the counters are reused per slab
  g_stats.nb_halo = ne;
  g_stats.n_zones = g.nz;
  g_stats.ra_bits = g.rb;
  g_stats.zone_height_arcsec = g.h_deg * 3600.0;

  // 3. A slabs through the cross-match; pairs leave through the ring
  int64_t total = 0;
  double compute_s = 0.0;  // device time of the slabs' cross-matches
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
  Caps caps = initial_caps(*dev, 2 * (uint64_t)SLAB, (uint64_t)half, true, false);
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
      HLC_TRY(hipEventRecord(sc.ev_t0, s));
      const int st = slab_match(*dev, A_ra[b] + u0, A_dec[b] + u0, (uint32_t)um, B, zstartB, g, r_arcsec, fp32,
                                caps, rp, rs, half, &found, o, s);
      HLC_TRY(hipEventRecord(sc.ev_t1, s));
      HLC_TRY(hipEventSynchronize(sc.ev_t1));
      compute_s += (double)elapsed(sc.ev_t0, sc.ev_t1) * 1e-3;
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
  if (compute_s > 0 && na > 0) dev->stream_rate = (double)na / compute_s;
  g_stats.n_pairs = total;
  *o->n_pairs = total;
  return HLC_OK;
}

}  // namespace
}  // namespace hlc

using namespace hlc;

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

}  // extern "C"
