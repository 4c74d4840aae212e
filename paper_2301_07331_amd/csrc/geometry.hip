// geometry.hip -- partition geometry of a call (Dec zones, RA bins, the
// frame of the data's footprint) and the thresholds of the decision.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "host.hpp"

namespace hlc {

// Smallest value >= v with at most 21 significant bits: b * (v / 2^rb) with
// b < 2^32 is then exact in FP64.
static double round_up_21(double v) {
  int e = 0;
  const double m = std::frexp(v, &e);
  return std::ldexp(std::ceil(std::ldexp(m, 20)), e - 20);
}

Geom make_geom(double r_arcsec, double h_as, int64_t na, int64_t nb, int ra_bits, const Frame& f) {
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

// Launches the footprint sample of a call; returns its sequence number for
// frame_finish.
unsigned long long frame_sample(Device& dev, const double* a_ra, const double* a_dec, int64_t na,
                                const double* b_ra, const double* b_dec, int64_t nb, hipStream_t s) {
  const unsigned long long seq = ++dev.fseq;
  launch_extent_sample(a_ra, a_dec, (uint32_t)na, b_ra, b_dec, (uint32_t)nb, dev.cnt, dev.fmsg_dev, seq, s);
  return seq;
}

bool quarter_sky(const Box& b) {
  const double d2r = M_PI / 180.0;
  return (std::sin(b.dhi * d2r) - std::sin(b.dlo * d2r)) * (b.rhi - b.rlo) * d2r > M_PI;
}

Frame frame_of_box(const Box& b) {
  Frame f;
  if (!b.any) return f;
  // a margin far above the rounding of the codes keeps every source inside
  const double m = 1e-9;
  f.dec_lo = std::max(-90.0, b.dlo - m);
  f.dec_hi = std::min(90.0, b.dhi + m);
  if (b.rhi - b.rlo < 170.0) {
    f.full_ra = false;
    f.ra_lo = b.rlo - m;
    f.ra_span = (b.rhi - b.rlo) + 2.0 * m;
  }
  return f;
}

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
  *out = frame_of_box(box());
  return HLC_OK;
}

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
  // chord of r for the FP32 filter, rounded up (the filter's own bound on its
  // rounding is added per A entry in the kernel)
  const double c_up = t.c_r * (1.0 + 8.0 * U64);
  float cf = (float)c_up;
  if ((double)cf < c_up) cf = std::nextafter(cf, INFINITY);
  t.c_r32 = cf;
  return t;
}

}  // namespace hlc
