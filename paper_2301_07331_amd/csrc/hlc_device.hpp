// hlc_device.hpp -- shared definitions of the gfx950 cross-match library:
// the partition geometry, degree-argument trigonometry, double-double
// arithmetic for threshold ties, and wave64 helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlc {

// ---------------------------------------------------------------------------
// Constants (double-double heads/tails printed by gen_constants.py).
// ---------------------------------------------------------------------------
constexpr double DEG2RAD_HI = 0x1.1df46a2529d39p-6;   // pi/180, head
constexpr double DEG2RAD_LO = 0x1.5c1d8becdd291p-62;  // pi/180, tail
constexpr double RAD2ARCSEC = 0x1.92dc67331ad7bp+17;  // 648000/pi rounded
constexpr double EPS_BAND = 1e-13;                    // FP64 haversine certification band
constexpr double TIE_REL = 1e-28;                     // double-double tie width
constexpr uint32_t HALO_BIT = 0x80000000u;            // B entry is a Dec-halo copy
constexpr uint32_t IDX_MASK = 0x7fffffffu;
constexpr int GROUP = 16;                             // A sources per group (one DPP row)
constexpr int MAXR = 4;                               // B ranges kept per group

// Partition geometry of one call: Dec zones of height h from dec0, RA bins
// of width ra_width from ra0 (the frame spans the data's footprint, or the
// whole sphere: dec0 = -90, ra0 = 0, nbins * ra_width = 360, full_ra); a
// source's key is ((zone << rb) | bin) << fb | frac, where frac is the
// position inside the bin in units of 2^-fb bin. Keys are sorted by (zone,
// bin) only; frac rides along and tightens the RA windows. Sources outside
// the frame are clamped into its edge cells (monotone, so still correct).
struct Geom {
  double h_deg;       // zone height between the polar cap bands (deg)
  double inv_h;       // 1 / h_deg
  double bin_scale;   // 1 / ra_width
  double dec0;        // Dec of the lower edge of zone 0
  double dec_s;       // lower edge of the first zone of height h_deg
  double dec_n;       // lower edge of the north cap band (nzn > 0)
  double hc_deg;      // zone height inside the cap bands
  double inv_hc;      // 1 / hc_deg
  int32_t nzs, nzn;   // zones of the south and north cap bands (0: none)
  double ra0;         // RA of the lower edge of bin 0
  double ra_width;    // bin width (deg)
  double r_deg;       // r_arcsec / 3600
  double rpad_deg;    // r padded outward for windows and halos
  int32_t nz;         // number of zones
  int32_t rb;         // RA bits; nbins = 1 << rb
  uint32_t nbins;
  int32_t fb;         // RA sub-bin bits carried in the low key bits (0..8)
  int32_t full_ra;    // the bins cover RA [0, 360): windows wrap at the seam
  int32_t frac_sorted;  // the sort also orders the sub-bin bits: B windows
                        // are searched at sub-bin resolution
};

// An entry count known on the host (base) plus an optional count that only
// the device knows yet (B halo copies appended by keygen), capped at the
// buffer capacity. Kernels read it instead of taking the count from the host,
// so a call needs no host round-trip before its sort and can be captured.
// Launch grids are sized from `cap`.
struct DevCount {
  uint32_t base, cap;
  const unsigned long long* extra;
  __device__ uint32_t get() const {
    unsigned long long v = (unsigned long long)base + (extra ? *extra : 0ull);
    return v < cap ? (uint32_t)v : cap;
  }
};

// Per-group B candidate ranges (positions in the sorted B arrays).
struct GroupRanges {
  uint32_t start[MAXR];
  uint32_t end[MAXR];
  uint32_t count;
  uint32_t pad_[3];
};

// Device-side counters, read back once per call.
struct Counters {
  unsigned long long n_halo;      // B halo copies appended by keygen
  unsigned long long n_pairs;     // pairs found (may exceed capacity)
  unsigned long long n_cand;      // filter survivors certified
  unsigned long long n_band;      // entries in the band list
  unsigned long long n_ties;      // decided in double-double
  unsigned int err;               // bit 0: bad coordinate in A, bit 1: in B
  unsigned int queue;             // work-queue head of persistent kernels
  unsigned long long aux[2];      // entry counts of multi-entry keygens (A, B)
  unsigned long long region_max;  // largest pair-region fill (compaction)
  unsigned long long cand_max;    // largest candidate-region fill
  // data footprint, each as a max of order-preserving codes of non-negative
  // doubles: ~code(dec + 90), code(dec + 90), ~code(ra), code(ra)
  unsigned long long ext[4];
};

struct Rec64 {      // FP64 working record (32 B)
  double x, y, z;
  uint32_t idx, pad;
};
struct Rec32 {      // batched form's FP32 working record (16 B): the unit
  float x, y, z;    // vector's offset from the job's frame centre, and the index
  uint32_t idx;
};

// FP32 working record of the single-call filter (16 B). The unit vector u
// (computed in FP64) is held as the corner of its FP32 lattice cell, each
// component rounded down to FP32 (x, y, z), and its offset inside that cell
// per axis as a fixed-point count of CELL_UNIT = 2^-34 (10 bits per axis in
// `off`: x in bits 0-9, y in 10-19, z in 20-29), rounded down. A cell is at
// most 2^-24 wide on an axis (|u_k| <= 1), so the count fits 10 bits and the
// stored position lies within 2^-34 of u on each axis, below it. The filter
// subtracts a group centre c (another lattice corner) from the corners and
// adds the scaled offsets, so it works in FP32 on small offsets from c
// instead of on unit vectors of magnitude 1.
struct CellRec32 {
  float x, y, z;
  uint32_t off;
};
constexpr float CELL_UNIT = 0x1p-34f;
constexpr double CELL_SCALE = 0x1p34;

// the cell record of a unit vector (FP64 components in [-1, 1])
__device__ inline CellRec32 encode_cell(double x, double y, double z) {
  CellRec32 r;
  r.x = __double2float_rd(x);
  r.y = __double2float_rd(y);
  r.z = __double2float_rd(z);
  // u - corner is exact in FP64 (below one FP32 ulp of u) and non-negative
  auto q = [](double u, float c) {
    const double t = floor((u - (double)c) * CELL_SCALE);
    return (uint32_t)(t < 1023.0 ? (t > 0.0 ? t : 0.0) : 1023.0);
  };
  r.off = q(x, r.x) | (q(y, r.y) << 10) | (q(z, r.z) << 20);
  return r;
}

// offset of a cell record from the centre (cx, cy, cz), in FP32:
// fl(fl(corner - c) + count * 2^-34) per axis
__device__ inline void cell_offset(const CellRec32& r, float cx, float cy, float cz, float& ox, float& oy,
                                   float& oz) {
  ox = fmaf((float)(r.off & 1023u), CELL_UNIT, r.x - cx);
  oy = fmaf((float)((r.off >> 10) & 1023u), CELL_UNIT, r.y - cy);
  oz = fmaf((float)(r.off >> 20), CELL_UNIT, r.z - cz);
}

// Logical block of a dispatched block such that consecutive logical blocks
// run on the same XCD (blocks are dispatched round-robin over the 8 XCDs, each
// with its own L2): neighbouring tiles then share that L2.
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
  const uint32_t q = nblocks >> 3, r = nblocks & 7u, x = bid & 7u, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// ---------------------------------------------------------------------------
// Geometry helpers (identical code for A and B keys, so they are monotone).
// ---------------------------------------------------------------------------
__host__ __device__ inline bool valid_pos(double ra, double dec) {
  // false for NaN as well
  return (ra >= 0.0) && (ra <= 360.0) && (dec >= -90.0) && (dec <= 90.0);
}

// Zones: nzs of height hc_deg from dec0 (south cap band), then zones of
// height h_deg from dec_s, then nzn of height hc_deg from dec_n (north cap
// band). Each band clamps to its own zones, so the map is monotone in dec.
__host__ __device__ inline int32_t zone_of(const Geom& g, double dec) {
  double t;
  int32_t base, top;
  if (g.nzs > 0 && dec < g.dec_s) {
    t = floor((dec - g.dec0) * g.inv_hc);
    base = 0;
    top = g.nzs - 1;
  } else if (g.nzn > 0 && dec >= g.dec_n) {
    t = floor((dec - g.dec_n) * g.inv_hc);
    base = g.nz - g.nzn;
    top = g.nz - 1;
  } else {
    t = floor((dec - g.dec_s) * g.inv_h);
    base = g.nzs;
    top = g.nz - g.nzn - 1;
  }
  if (!(t >= 0.0)) return base;
  if (t > (double)(top - base)) return top;
  return base + (int32_t)t;
}

// lower edge and height of zone z
__host__ __device__ inline double zone_lo(const Geom& g, int32_t z) {
  if (z < g.nzs) return g.dec0 + (double)z * g.hc_deg;
  if (z >= g.nz - g.nzn) return g.dec_n + (double)(z - (g.nz - g.nzn)) * g.hc_deg;
  return g.dec_s + (double)(z - g.nzs) * g.h_deg;
}
__host__ __device__ inline double zone_height(const Geom& g, int32_t z) {
  return (z < g.nzs || z >= g.nz - g.nzn) ? g.hc_deg : g.h_deg;
}

__host__ __device__ inline uint32_t bin_of(const Geom& g, double ra) {
  double t = floor((ra - g.ra0) * g.bin_scale);
  if (!(t >= 0.0)) return 0u;
  if (t > (double)(g.nbins - 1)) return g.nbins - 1;
  return (uint32_t)t;
}

// position inside bin b of an RA with bin_of(g, ra) == b, in [0, 2^fb):
// floor(((ra - ra0) * scale - b) * 2^fb), so (ra - ra0) * scale >= b + frac / 2^fb
__host__ __device__ inline uint32_t frac_of(const Geom& g, double ra, uint32_t b) {
  const double t = ((ra - g.ra0) * g.bin_scale - (double)b) * (double)(1u << g.fb);
  const double f = floor(t);
  const double top = (double)((1u << g.fb) - 1u);
  return f >= 0.0 ? (uint32_t)(f < top ? f : top) : 0u;
}
// key of (zone z, bin b) with frac 0: the smallest key of the cell
__host__ __device__ inline uint32_t make_key(const Geom& g, int32_t z, uint32_t b) {
  return (((uint32_t)z << g.rb) | b) << g.fb;
}
__host__ __device__ inline int32_t key_zone(const Geom& g, uint32_t k) { return (int32_t)(k >> (g.rb + g.fb)); }
__host__ __device__ inline uint32_t key_bin(const Geom& g, uint32_t k) { return (k >> g.fb) & (g.nbins - 1); }
__host__ __device__ inline uint32_t key_frac(const Geom& g, uint32_t k) { return k & ((1u << g.fb) - 1u); }
__host__ __device__ inline bool same_zone(const Geom& g, uint32_t ka, uint32_t kb) {
  return ((ka ^ kb) >> (g.rb + g.fb)) == 0u;
}

// ---------------------------------------------------------------------------
// sin and cos of r, |r| <= pi/4, from their Taylor series through r^17 and
// r^16 in Horner form (the omitted terms are below 2^-62 and 2^-58 of the
// results). Every step is one explicit FMA or product, so the rounding is
// the same wherever the sequence is replayed; the error is below 1.5 ulp
// (checked against a 60-digit evaluation of the same arguments on the CPU).
// ---------------------------------------------------------------------------
__host__ __device__ inline void sincos_small(double r, double* s, double* c) {
  const double z = r * r;
  double ps = 1.0 / 355687428096000.0;  // 1/17!
  ps = fma(ps, z, -1.0 / 1307674368000.0);
  ps = fma(ps, z, 1.0 / 6227020800.0);
  ps = fma(ps, z, -1.0 / 39916800.0);
  ps = fma(ps, z, 1.0 / 362880.0);
  ps = fma(ps, z, -1.0 / 5040.0);
  ps = fma(ps, z, 1.0 / 120.0);
  ps = fma(ps, z, -1.0 / 6.0);
  *s = fma(ps, z * r, r);
  double pc = 1.0 / 20922789888000.0;  // 1/16!
  pc = fma(pc, z, -1.0 / 87178291200.0);
  pc = fma(pc, z, 1.0 / 479001600.0);
  pc = fma(pc, z, -1.0 / 3628800.0);
  pc = fma(pc, z, 1.0 / 40320.0);
  pc = fma(pc, z, -1.0 / 720.0);
  pc = fma(pc, z, 1.0 / 24.0);
  pc = fma(pc, z, -0.5);
  *c = fma(pc, z, 1.0);
}

// ---------------------------------------------------------------------------
// sin and cos of an angle in degrees, |x| <= 360.
// The argument is reduced by the nearest multiple of 90 degrees, which is
// exact in FP64 for |x| <= 360 (Sterbenz), converted to radians with a
// double-double pi/180, and the quadrant is applied by swapping/negating:
// quadrant q gives (sin, cos) = (sr, cr), (cr, -sr), (-sr, -cr), (-cr, sr)
// for q = 0, 1, 2, 3 (selects, no branches: the quadrants of a wave's
// lanes differ).
// ---------------------------------------------------------------------------
__device__ inline void sincos_deg(double x, double* s, double* c) {
  double q = rint(x * (1.0 / 90.0));
  double y = fma(-q, 90.0, x);
  double p = y * DEG2RAD_HI;
  double e = fma(y, DEG2RAD_HI, -p);
  double r = p + fma(y, DEG2RAD_LO, e);
  double sr, cr;
  sincos_small(r, &sr, &cr);
  const int qi = ((int)q) & 3;
  const double s0 = (qi & 1) ? cr : sr;
  const double c0 = (qi & 1) ? sr : cr;
  *s = (qi & 2) ? -s0 : s0;
  *c = ((qi + 1) & 2) ? -c0 : c0;
}

// unit vector of (ra, dec) in degrees; the keygen and the FP32 filter of a
// side read in place use this one sequence, so their cell records agree
__device__ inline void unit_vector(double ra, double dec, double& x, double& y, double& z) {
  double sd, cd, sa, ca;
  sincos_deg(dec, &sd, &cd);
  sincos_deg(ra, &sa, &ca);
  x = cd * ca;
  y = cd * sa;
  z = sd;
}

__device__ inline double cos_deg_abs(double dec) {
  // cos of a declination, relatively accurate near the poles
  double a = fabs(dec);
  double s, c;
  if (a <= 45.0) { sincos_deg(a, &s, &c); return c; }
  sincos_deg(90.0 - a, &s, &c);
  return s;
}

// RA difference folded into [-180, 180] without an extra rounding: the
// larger value is first reduced by 360 (exact for values in [180, 360]).
__device__ inline double dra_fold(double ra1, double ra2) {
  if (fabs(ra1 - ra2) > 180.0) {
    if (ra1 > ra2) ra1 -= 360.0; else ra2 -= 360.0;
  }
  return ra1 - ra2;
}

// Haversine h = sin^2(theta/2) in FP64 from degrees.
__device__ inline double haversine64(double ra1, double dec1, double ra2, double dec2) {
  double s1, c1, s2, c2;
  sincos_deg(0.5 * (dec1 - dec2), &s1, &c1);
  sincos_deg(0.5 * dra_fold(ra1, ra2), &s2, &c2);
  return s1 * s1 + cos_deg_abs(dec1) * cos_deg_abs(dec2) * (s2 * s2);
}

// ---------------------------------------------------------------------------
// HEALPix nested pixel index at Nside = 2^order (the paper's first-level
// partition, section 4.2), from the definitions of the pixelisation: twelve
// base faces; in the equatorial zone |z| <= 2/3 the in-face coordinates come
// from two families of straight lines in (phi, z), in the polar caps from
// lines scaled by sqrt(1 - |z|); the nested index interleaves their bits.
// ---------------------------------------------------------------------------
__device__ inline uint32_t hp_spread(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ inline uint32_t hp_nest(int order, double ra, double dec) {
  const int32_t ns = 1 << order;
  double z, c;
  sincos_deg(dec, &z, &c);
  const double za = fabs(z);
  double tt = ra * (1.0 / 90.0);
  if (tt >= 4.0) tt -= 4.0;
  if (tt < 0.0) tt += 4.0;
  int32_t face, ix, iy;
  if (za <= 2.0 / 3.0) {
    const double t1 = ns * (0.5 + tt), t2 = ns * (z * 0.75);
    const int32_t jp = (int32_t)(t1 - t2), jm = (int32_t)(t1 + t2);
    const int32_t ifp = jp >> order, ifm = jm >> order;
    face = (ifp == ifm) ? (ifp | 4) : (ifp < ifm ? ifp : ifm + 8);
    ix = jm & (ns - 1);
    iy = ns - (jp & (ns - 1)) - 1;
  } else {
    int32_t ntt = (int32_t)tt;
    if (ntt > 3) ntt = 3;
    const double tp = tt - (double)ntt;
    double sh, ch;  // 1 - |z| = 2 sin^2(colatitude / 2)
    sincos_deg(0.5 * (90.0 - fabs(dec)), &sh, &ch);
    const double tmp = ns * 2.449489742783178 * sh;  // sqrt(6)
    int32_t jp = (int32_t)(tp * tmp), jm = (int32_t)((1.0 - tp) * tmp);
    jp = min(jp, ns - 1);
    jm = min(jm, ns - 1);
    if (z >= 0.0) {
      face = ntt;
      ix = ns - jm - 1;
      iy = ns - jp - 1;
    } else {
      face = ntt + 8;
      ix = jp;
      iy = jm;
    }
  }
  return (uint32_t)face * (uint32_t)ns * (uint32_t)ns + (hp_spread((uint32_t)ix) | (hp_spread((uint32_t)iy) << 1));
}

// Distinct pixels of a record under the quad-direction strategy (section
// 3.2, Algorithm 1 read with its Dec-minus line as dec - R): its own pixel
// and those of (ra +- R, dec) and (ra, dec +- R); RA wraps, Dec stops at +-90.
__device__ inline int hp_quad(int order, double ra, double dec, double R, uint32_t out[5]) {
  int n = 0;
  auto put = [&](uint32_t p) {
    for (int k = 0; k < n; ++k)
      if (out[k] == p) return;
    out[n++] = p;
  };
  double rp = ra + R, rm = ra - R;
  if (rp >= 360.0) rp -= 360.0;
  if (rm < 0.0) rm += 360.0;
  put(hp_nest(order, ra, dec));
  put(hp_nest(order, rp, dec));
  put(hp_nest(order, rm, dec));
  put(hp_nest(order, ra, fmin(dec + R, 90.0)));
  put(hp_nest(order, ra, fmax(dec - R, -90.0)));
  return n;
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (value = hi + lo, |lo| <= ulp(hi)/2).
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ inline dd quick_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ inline dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__device__ inline dd dd_mul(dd x, dd y) {
  double p = x.hi * y.hi;
  double e = fma(x.hi, y.hi, -p);
  e = fma(x.hi, y.lo, e);
  e = fma(x.lo, y.hi, e);
  return quick_two_sum(p, e);
}
__device__ inline dd dd_mul_d(dd x, double y) {
  double p = x.hi * y;
  double e = fma(x.hi, y, -p);
  e = fma(x.lo, y, e);
  return quick_two_sum(p, e);
}
// x / n for an exactly representable n
__device__ inline dd dd_div_d(dd x, double n) {
  double q1 = x.hi / n;
  double p = q1 * n;
  double pe = fma(q1, n, -p);
  dd r = dd_add(x, dd{-p, -pe});
  double q2 = r.hi / n;
  return quick_two_sum(q1, q2);
}

// sin and cos of a double-double angle in radians, |x| <= pi/2 + small.
__device__ inline dd dd_sin(dd x) {
  dd x2 = dd_mul(x, x);
  dd term = x, sum = x;
  for (int k = 1; k < 40; ++k) {
    term = dd_div_d(dd_mul(term, x2), (double)((2 * k) * (2 * k + 1)));
    term = dd_neg(term);
    sum = dd_add(sum, term);
    if (fabs(term.hi) <= 1e-36 * fabs(sum.hi)) break;
  }
  return sum;
}
__device__ inline dd dd_cos(dd x) {
  dd x2 = dd_mul(x, x);
  dd term = {1.0, 0.0}, sum = {1.0, 0.0};
  for (int k = 1; k < 40; ++k) {
    term = dd_div_d(dd_mul(term, x2), (double)((2 * k - 1) * (2 * k)));
    term = dd_neg(term);
    sum = dd_add(sum, term);
    if (fabs(term.hi) <= 1e-36 * fabs(sum.hi)) break;
  }
  return sum;
}
__device__ inline dd dd_deg2rad(dd d) { return dd_mul(d, dd{DEG2RAD_HI, DEG2RAD_LO}); }

// cos(dec) in double-double, relatively accurate near the poles.
__device__ inline dd dd_cos_dec(double dec) {
  double a = fabs(dec);
  if (a <= 45.0) return dd_cos(dd_deg2rad(dd{a, 0.0}));
  return dd_sin(dd_deg2rad(dd{90.0 - a, 0.0}));  // 90 - a exact
}

// Haversine in double-double.
__device__ inline dd haversine_dd(double ra1, double dec1, double ra2, double dec2) {
  dd ddec = two_sum(dec1, -dec2);
  double a = ra1, b = ra2;
  if (fabs(a - b) > 180.0) {
    if (a > b) a -= 360.0; else b -= 360.0;  // exact
  }
  dd dra = two_sum(a, -b);
  dd s1 = dd_sin(dd_mul_d(dd_deg2rad(ddec), 0.5));
  dd s2 = dd_sin(dd_mul_d(dd_deg2rad(dra), 0.5));
  dd cc = dd_mul(dd_cos_dec(dec1), dd_cos_dec(dec2));
  return dd_add(dd_mul(s1, s1), dd_mul(cc, dd_mul(s2, s2)));
}

__device__ inline dd dd_sqrt(dd x) {
  if (!(x.hi > 0.0)) return {0.0, 0.0};
  const double r = sqrt(x.hi);
  const double p = r * r;
  const double pe = fma(r, r, -p);
  const dd d = dd_add(x, dd{-p, -pe});
  return quick_two_sum(r, d.hi / (2.0 * r));
}

// sin^2(r/2) for the eq. (4) radius r = k sqrt(ea^2 + eb^2) arcsec, in
// double-double.
__device__ inline dd threshold_pair_dd(double k, double ea, double eb) {
  const dd ea2 = dd_mul(dd{ea, 0.0}, dd{ea, 0.0});
  const dd eb2 = dd_mul(dd{eb, 0.0}, dd{eb, 0.0});
  const dd r_as = dd_mul_d(dd_sqrt(dd_add(ea2, eb2)), k);
  const dd r = dd_div_d(r_as, 3600.0);
  const dd s = dd_sin(dd_mul_d(dd_deg2rad(r), 0.5));
  return dd_mul(s, s);
}

// sin^2(r/2) with r = r_arcsec / 3600 degrees, in double-double.
__device__ inline dd threshold_dd(double r_arcsec) {
  dd r = dd_div_d(dd{r_arcsec, 0.0}, 3600.0);
  dd s = dd_sin(dd_mul_d(dd_deg2rad(r), 0.5));
  return dd_mul(s, s);
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ inline uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of mask below this lane
__device__ inline uint32_t rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// At most MAXR ascending B ranges, kept in registers (every index below is
// static): a range touching or overlapping the last one extends it; one
// more than MAXR is merged across the smallest gap. Merging only adds B
// entries of the window's neighbourhood (other-zone entries are dropped by
// the filter), so the ranges still cover every candidate.
struct RangeList {
  uint32_t s[MAXR + 1];
  uint32_t e[MAXR + 1];
  int n;
  __device__ void clear() {
    n = 0;
#pragma unroll
    for (int i = 0; i <= MAXR; ++i) s[i] = e[i] = 0u;
  }
  __device__ void add(uint32_t a, uint32_t b) {
    if (a >= b) return;
    bool merged = false;
#pragma unroll
    for (int i = 0; i < MAXR; ++i)
      if (i == n - 1 && a <= e[i]) {  // overlapping or touching the previous one
        e[i] = max(e[i], b);
        merged = true;
      }
    if (merged) return;
#pragma unroll
    for (int i = 0; i <= MAXR; ++i)
      if (i == n) {
        s[i] = a;
        e[i] = b;
      }
    ++n;
    if (n <= MAXR) return;
    int best = 0;
    uint32_t gap = s[1] - e[0];
#pragma unroll
    for (int i = 1; i < MAXR; ++i)
      if (s[i + 1] - e[i] < gap) {
        gap = s[i + 1] - e[i];
        best = i;
      }
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
      if (i == best) e[i] = e[i + 1];
      if (i > best) {
        s[i] = s[i + 1];
        e[i] = e[i + 1];
      }
    }
    n = MAXR;
  }
};

// Broadcast lane n of each 16-lane row to the whole row (DPP row_newbcast).
// Every lane has a valid source, so the zero "old" value is never seen; it
// lets the compiler fold the broadcast into the VALU op that consumes it
// (v_sub_f32_dpp instead of v_mov_b32_dpp + v_sub_f32).
template <int N>
__device__ inline float row_bcast(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + N, 0xf, 0xf, true));
}
template <int N>
__device__ inline uint32_t row_bcast_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + N, 0xf, 0xf, true);
}
template <int N>
__device__ inline double row_bcast(double v) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x150 + N, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x150 + N, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

}  // namespace hlc
