// oracle.cpp -- CPU reference for the positional cross-match.
//
// TEST INFRASTRUCTURE ONLY. Only tests/, the smoke entry point and the CPU
// baseline leg of bench.py may load this library. It shares no code, header,
// constant or table with the HIP library under paper_2301_07331_amd/.
//
// What it computes (paper, section 2.1):
//   Two catalogues A, B of (RA, Dec) positions in degrees and a threshold r.
//   The angular separation of two positions is the great-circle angle of
//   eq. (1). A pair matches when that angle does not exceed the threshold
//   (eq. (4) uses an inclusive "<="), and every matching pair is reported
//   (section 2.1 counts all m*n comparisons; section 4.3.2 keeps a result for
//   every catalogue pair). Here the threshold is a single radius given in
//   arcseconds, r = r_arcsec / 3600 degrees read as an exact real, and the
//   inputs are read as exact reals too:
//
//     S(A, B, r) = { (i, j) : theta(A_i, B_j) <= r }.
//
// How:
//   * The separation is evaluated with the haversine form of eq. (1)'s
//     quantity, h = sin^2(dDec/2) + cos(Dec_i) cos(Dec_j) sin^2(dRA/2),
//     theta = 2 asin(sqrt(h)). (Eq. (1) itself loses about half the digits of
//     a 1-arcsec angle in FP64; eq. (3) is a flat-sky approximation that is
//     wrong near the poles and across the RA seam. Neither is used.)
//   * Decision: h is compared with H = sin^2(r/2) in FP64. Outside a relative
//     band of EPS_BAND around H the FP64 answer is certain (bound derived at
//     EPS_BAND below); inside it the same formula is re-evaluated in IEEE
//     binary128 (libquadmath). A binary128 result within 1e-28 H of H is
//     treated as a true tie and counted as a match ("<=").
//   * Candidates come from a plain declination-zone join (the Zones scheme the
//     paper lists among sky indexes in section 2.2): B is sorted by
//     (zone, RA); each A_i visits the zones its Dec +- r window touches and,
//     in each, the RA window of half-width asin(sin r / cos Dec_i) (the exact
//     largest RA offset of a small circle of radius r), split at the 0/360
//     seam and widened to the whole zone within r of a pole. The windows are
//     padded outward so that FP64 rounding can only add candidates. The
//     brute-force entry point runs the same decision over all m*n pairs; the
//     tests use it to show the zone join misses nothing.
//
// Domain: RA in [0, 360], Dec in [-90, 90], finite; RA 360 is the same point
// as RA 0. Indices are uint32 (n < 2^31). Invalid input returns -1.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <omp.h>
#include <parallel/algorithm>
#include <quadmath.h>

namespace {

typedef __float128 quad;

// ---------------------------------------------------------------------------
// FP64 error budget for h and H (u = 2^-53).
//   dDec = fl(Dec_i - Dec_j): rel. err <= u (exact when Sterbenz applies).
//   dRA: the larger RA is first reduced by 360 when |RA_i - RA_j| > 180; that
//        reduction is exact (Sterbenz, RA in [180, 360]); the difference then
//        has rel. err <= u.
//   x = fl(fl(d * K) * 0.5), K = fl(pi/180): rel. err <= 3u.
//   s = sin(x): with |x| <= pi/2, |x cot x| <= 1, so rel. err <= 3u + 2u
//        (glibc sin/cos are within 1 ulp; 2u is assumed).
//   cos(Dec): cos(fl(Dec*K)) for |Dec| <= 45 (rel. err <= 2u*tan(pi/4) + 2u),
//        sin(fl((90-|Dec|)*K)) above 45 (90-|Dec| exact; rel. err <= 4u).
//   h = s1^2 + cos_i cos_j s2^2: both terms >= 0, rel. err <= 22u.
//   H = sin(fl(fl(r_arcsec/3600)*K)/2)^2: rel. err <= 11u.
//   Deciding h < H(1-eps) or h > H(1+eps) is therefore certain when
//   eps >= 22u + 11u + 2u = 35u ~= 3.9e-15. EPS_BAND is over 25x that.
constexpr double U64 = 1.1102230246251565e-16;
constexpr double EPS_BAND = 1e-13;
static_assert(EPS_BAND >= 20.0 * 35.0 * U64, "band narrower than 20x the FP64 error bound");
constexpr double TIE_REL = 1e-28;
constexpr double K64 = M_PI / 180.0;
constexpr double RAD2AS = 648000.0 / M_PI;

bool valid_pos(double ra, double dec) {
  return std::isfinite(ra) && std::isfinite(dec) && ra >= 0.0 && ra <= 360.0 &&
         dec >= -90.0 && dec <= 90.0;
}

double cos_dec64(double dec) {
  double a = std::fabs(dec);
  return a <= 45.0 ? std::cos(a * K64) : std::sin((90.0 - a) * K64);
}

// RA difference folded into [-180, 180] without an extra rounding.
double dra64(double ra1, double ra2) {
  if (std::fabs(ra1 - ra2) > 180.0) {
    if (ra1 > ra2) ra1 -= 360.0; else ra2 -= 360.0;
  }
  return ra1 - ra2;
}

quad cos_decq(double dec) {
  quad Kq = M_PIq / 180;
  quad a = fabsq((quad)dec);
  return a <= 45 ? cosq(a * Kq) : sinq((90 - a) * Kq);
}

quad drag(double ra1, double ra2) {
  quad a = ra1, b = ra2;
  if (fabsq(a - b) > 180) {
    if (a > b) a -= 360; else b -= 360;
  }
  return a - b;
}

struct Thresh {
  double r_deg;      // fl(r_arcsec / 3600)
  double H;          // sin^2(r/2), FP64
  quad Hq;           // sin^2(r/2), binary128, r = r_arcsec/3600 in binary128
};

Thresh make_thresh(double r_arcsec) {
  Thresh t;
  t.r_deg = r_arcsec / 3600.0;
  double s = std::sin(t.r_deg * K64 * 0.5);
  t.H = s * s;
  quad rq = (quad)r_arcsec / 3600;
  quad sq = sinq(rq * (M_PIq / 180) / 2);
  t.Hq = sq * sq;
  return t;
}

// Outcome of one pair decision.
enum { OUT = 0, IN_FP64 = 1, IN_QUAD = 2, IN_TIE = 3, OUT_QUAD = 4 };

// Decide theta(p1, p2) <= r and give the separation in arcsec when it holds.
int decide(double ra1, double dec1, double cd1, double ra2, double dec2, double cd2,
           const Thresh& t, double* sep_as) {
  double ddec = dec1 - dec2;
  double dra = dra64(ra1, ra2);
  double s1 = std::sin(ddec * K64 * 0.5);
  double s2 = std::sin(dra * K64 * 0.5);
  double h = s1 * s1 + cd1 * cd2 * (s2 * s2);
  if (h < t.H * (1.0 - EPS_BAND)) {
    *sep_as = 2.0 * std::asin(std::sqrt(h)) * RAD2AS;
    return IN_FP64;
  }
  if (h > t.H * (1.0 + EPS_BAND)) return OUT;
  // Band: binary128 re-evaluation of the same quantity.
  quad Kq = M_PIq / 180;
  quad ddq = (quad)dec1 - (quad)dec2;
  quad draq = drag(ra1, ra2);
  quad q1 = sinq(ddq * Kq / 2);
  quad q2 = sinq(draq * Kq / 2);
  quad hq = q1 * q1 + cos_decq(dec1) * cos_decq(dec2) * (q2 * q2);
  quad diff = hq - t.Hq;
  if (diff > TIE_REL * t.Hq) return OUT_QUAD;
  *sep_as = (double)(2 * asinq(sqrtq(hq)) * (648000 / M_PIq));
  return fabsq(diff) <= TIE_REL * t.Hq ? IN_TIE : IN_QUAD;
}

// Per-pair threshold of eq. (4): r_ij = k * sqrt(ea_i^2 + eb_j^2) arcsec.
// H = sin^2(r_ij / 2) in FP64 has a relative error of a few u (sqrt and the
// products add < 4u to the 11u of make_thresh), inside the same EPS_BAND.
Thresh thresh_pair(double k, double ea, double eb) {
  Thresh t;
  double r_as = k * std::sqrt(ea * ea + eb * eb);
  t.r_deg = r_as / 3600.0;
  double s = std::sin(t.r_deg * K64 * 0.5);
  t.H = s * s;
  quad rq = (quad)k * sqrtq((quad)ea * (quad)ea + (quad)eb * (quad)eb) / 3600;
  quad sq = sinq(rq * (M_PIq / 180) / 2);
  t.Hq = sq * sq;
  return t;
}

struct Hit {
  uint32_t a, b;
  double sep;
};

struct Stats {
  int64_t candidates = 0, band = 0, ties = 0;
};

}  // namespace

struct oracle_result {
  std::vector<Hit> hits;
  Stats st;
};

namespace {

bool check_inputs(const double* ra, const double* dec, int64_t n) {
  bool ok = true;
#pragma omp parallel for reduction(&& : ok) schedule(static)
  for (int64_t i = 0; i < n; ++i) ok = ok && valid_pos(ra[i], dec[i]);
  return ok;
}

void finish(oracle_result* res, std::vector<std::vector<Hit>>& parts, bool sort_pairs) {
  size_t tot = 0;
  for (auto& p : parts) tot += p.size();
  res->hits.reserve(tot);
  for (auto& p : parts) res->hits.insert(res->hits.end(), p.begin(), p.end());
  if (sort_pairs)
    __gnu_parallel::sort(res->hits.begin(), res->hits.end(), [](const Hit& x, const Hit& y) {
      return x.a != y.a ? x.a < y.a : x.b < y.b;
    });
}

int resolve_threads(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

}  // namespace

extern "C" {

int oracle_abi_version(void) { return 1; }

// Single pair: returns the outcome code (0 out, 1 in by FP64, 2 in after the
// binary128 re-evaluation, 3 in as a true tie, 4 out after binary128) and
// the separation (arcsec) when in; -1 on invalid input.
int oracle_pair(double ra1, double dec1, double ra2, double dec2, double r_arcsec,
                double* sep_arcsec) {
  if (!valid_pos(ra1, dec1) || !valid_pos(ra2, dec2) || !(r_arcsec > 0.0)) return -1;
  Thresh t = make_thresh(r_arcsec);
  double sep = NAN;
  int k = decide(ra1, dec1, cos_dec64(dec1), ra2, dec2, cos_dec64(dec2), t, &sep);
  if (sep_arcsec) *sep_arcsec = sep;
  return k;
}

// Separation in arcsec evaluated entirely in binary128 (haversine), rounded
// once to FP64. Used by the tests as the high-precision value.
double oracle_sep_q(double ra1, double dec1, double ra2, double dec2) {
  quad Kq = M_PIq / 180;
  quad q1 = sinq(((quad)dec1 - (quad)dec2) * Kq / 2);
  quad q2 = sinq(drag(ra1, ra2) * Kq / 2);
  quad hq = q1 * q1 + cos_decq(dec1) * cos_decq(dec2) * (q2 * q2);
  return (double)(2 * asinq(sqrtq(hq)) * (648000 / M_PIq));
}

// Exact-real decision of theta <= r evaluated in binary128 only: 1 in, 0 out.
int oracle_pair_q(double ra1, double dec1, double ra2, double dec2, double r_arcsec) {
  quad Kq = M_PIq / 180;
  quad q1 = sinq(((quad)dec1 - (quad)dec2) * Kq / 2);
  quad q2 = sinq(drag(ra1, ra2) * Kq / 2);
  quad hq = q1 * q1 + cos_decq(dec1) * cos_decq(dec2) * (q2 * q2);
  quad sr = sinq((quad)r_arcsec / 3600 * Kq / 2);
  quad Hq = sr * sr;
  return hq - Hq <= TIE_REL * Hq ? 1 : 0;
}

// Zone join. On success returns a result handle (caller frees it);
// *status = 0, or -1 for invalid input (handle is NULL).
oracle_result* oracle_xmatch(const double* a_ra, const double* a_dec, int64_t na,
                             const double* b_ra, const double* b_dec, int64_t nb,
                             double r_arcsec, int nthreads, int sort_pairs, int* status) {
  *status = -1;
  if (na < 0 || nb < 0 || na >= (int64_t(1) << 31) || nb >= (int64_t(1) << 31)) return nullptr;
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return nullptr;
  int nt = resolve_threads(nthreads);
  omp_set_num_threads(nt);
  if (!check_inputs(a_ra, a_dec, na) || !check_inputs(b_ra, b_dec, nb)) return nullptr;
  auto* res = new oracle_result();
  *status = 0;
  if (na == 0 || nb == 0) return res;

  Thresh t = make_thresh(r_arcsec);
  // Outward-padded radius for the candidate windows (degrees).
  const double rp = t.r_deg * (1.0 + 1e-9) + 1e-12;
  // Zone height = r, capped at 2^22 zones.
  const double zh = std::max(t.r_deg, 180.0 / double(1 << 22));
  const int64_t nz = (int64_t)std::ceil(180.0 / zh);
  auto zone_of = [&](double dec) -> int64_t {
    int64_t z = (int64_t)std::floor((dec + 90.0) / zh);
    return std::min<int64_t>(std::max<int64_t>(z, 0), nz - 1);
  };

  // B sorted by (zone, RA).
  struct BRec {
    int64_t zone;
    double ra, dec, cd;
    uint32_t idx;
  };
  std::vector<BRec> B(nb);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nb; ++j)
    B[j] = BRec{zone_of(b_dec[j]), b_ra[j], b_dec[j], cos_dec64(b_dec[j]), (uint32_t)j};
  __gnu_parallel::sort(B.begin(), B.end(), [](const BRec& x, const BRec& y) {
    if (x.zone != y.zone) return x.zone < y.zone;
    if (x.ra != y.ra) return x.ra < y.ra;
    return x.idx < y.idx;
  });
  std::vector<int64_t> zstart(nz + 1, 0);
  for (int64_t j = 0; j < nb; ++j) zstart[B[j].zone + 1]++;
  for (int64_t z = 0; z < nz; ++z) zstart[z + 1] += zstart[z];

  std::vector<std::vector<Hit>> parts(nt);
  std::vector<Stats> tst(nt);
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
    auto& out = parts[tid];
    auto& st = tst[tid];
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < na; ++i) {
      const double ra = a_ra[i], dec = a_dec[i], cd = cos_dec64(dec);
      // RA half-width of the window, degrees; >= 180 means the whole zone.
      double w = 180.0;
      if (std::fabs(dec) + rp < 90.0) {
        double x = std::sin(rp * K64) / cd;
        if (x < 0.99) w = std::asin(x) / K64 * (1.0 + 1e-9) + 1e-12;
      }
      double lo[2], hi[2];
      int nint = 0;
      if (w >= 180.0) {
        lo[0] = 0.0; hi[0] = 360.0; nint = 1;
      } else if (ra - w < 0.0) {
        lo[0] = 0.0; hi[0] = ra + w;
        lo[1] = ra - w + 360.0; hi[1] = 360.0; nint = 2;
      } else if (ra + w > 360.0) {
        lo[0] = ra - w; hi[0] = 360.0;
        lo[1] = 0.0; hi[1] = ra + w - 360.0; nint = 2;
      } else {
        lo[0] = ra - w; hi[0] = ra + w; nint = 1;
      }
      const int64_t z0 = zone_of(dec - rp), z1 = zone_of(dec + rp);
      for (int64_t z = z0; z <= z1; ++z) {
        auto zb = B.begin() + zstart[z], ze = B.begin() + zstart[z + 1];
        for (int k = 0; k < nint; ++k) {
          auto it = std::lower_bound(zb, ze, lo[k], [](const BRec& b, double v) { return b.ra < v; });
          for (; it != ze && it->ra <= hi[k]; ++it) {
            ++st.candidates;
            double sep;
            int o = decide(ra, dec, cd, it->ra, it->dec, it->cd, t, &sep);
            if (o == IN_QUAD || o == IN_TIE || o == OUT_QUAD) ++st.band;
            if (o == IN_TIE) ++st.ties;
            if (o == IN_FP64 || o == IN_QUAD || o == IN_TIE) out.push_back(Hit{(uint32_t)i, it->idx, sep});
          }
        }
      }
    }
  }
  for (auto& s : tst) {
    res->st.candidates += s.candidates;
    res->st.band += s.band;
    res->st.ties += s.ties;
  }
  finish(res, parts, sort_pairs != 0);
  return res;
}

// Per-source error radii (eq. (4)): pairs with theta <= k sqrt(ea_i^2 + eb_j^2)
// arcsec. Candidates come from the zone join at the largest such radius;
// `brute` != 0 runs all m*n pairs instead.
oracle_result* oracle_xmatch_radii(const double* a_ra, const double* a_dec, const double* a_err,
                                   int64_t na, const double* b_ra, const double* b_dec,
                                   const double* b_err, int64_t nb, double k, int nthreads, int brute,
                                   int* status) {
  *status = -1;
  if (na < 0 || nb < 0 || na >= (int64_t(1) << 31) || nb >= (int64_t(1) << 31)) return nullptr;
  if (!(k > 0.0) || !std::isfinite(k)) return nullptr;
  int nt = resolve_threads(nthreads);
  omp_set_num_threads(nt);
  if (!check_inputs(a_ra, a_dec, na) || !check_inputs(b_ra, b_dec, nb)) return nullptr;
  double ea_max = 0.0, eb_max = 0.0;
  for (int64_t i = 0; i < na; ++i) {
    if (!(a_err[i] >= 0.0) || !std::isfinite(a_err[i])) return nullptr;
    ea_max = std::max(ea_max, a_err[i]);
  }
  for (int64_t j = 0; j < nb; ++j) {
    if (!(b_err[j] >= 0.0) || !std::isfinite(b_err[j])) return nullptr;
    eb_max = std::max(eb_max, b_err[j]);
  }
  const double rmax = k * std::sqrt(ea_max * ea_max + eb_max * eb_max) * (1.0 + 1e-12);
  if (!(rmax <= 3600.0)) return nullptr;
  auto* res = new oracle_result();
  *status = 0;
  if (na == 0 || nb == 0) return res;
  std::vector<std::vector<Hit>> parts(nt);
  std::vector<Stats> tst(nt);
  auto one = [&](int tid, int64_t i, int64_t j) {
    const Thresh t = thresh_pair(k, a_err[i], b_err[j]);  // H = 0 keeps identical points
    double sep;
    int o = decide(a_ra[i], a_dec[i], cos_dec64(a_dec[i]), b_ra[j], b_dec[j], cos_dec64(b_dec[j]), t, &sep);
    ++tst[tid].candidates;
    if (o == IN_QUAD || o == IN_TIE || o == OUT_QUAD) ++tst[tid].band;
    if (o == IN_TIE) ++tst[tid].ties;
    if (o == IN_FP64 || o == IN_QUAD || o == IN_TIE) parts[tid].push_back(Hit{(uint32_t)i, (uint32_t)j, sep});
  };
  if (brute) {
#pragma omp parallel num_threads(nt)
    {
      int tid = omp_get_thread_num();
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j) one(tid, i, j);
    }
  } else {
    // candidates from the zone join at rmax (its pairs are a superset)
    int st2 = 0;
    // (with all errors zero only identical points match; any positive join
    // radius finds them)
    oracle_result* cand = oracle_xmatch(a_ra, a_dec, na, b_ra, b_dec, nb, std::max(rmax, 1e-6), nt, 0, &st2);
    if (!cand) {
      delete res;
      *status = -1;
      return nullptr;
    }
    const int64_t nc = (int64_t)cand->hits.size();
#pragma omp parallel num_threads(nt)
    {
      int tid = omp_get_thread_num();
#pragma omp for schedule(static)
      for (int64_t c = 0; c < nc; ++c) one(tid, cand->hits[c].a, cand->hits[c].b);
    }
    delete cand;
  }
  for (auto& st : tst) {
    res->st.candidates += st.candidates;
    res->st.band += st.band;
    res->st.ties += st.ties;
  }
  finish(res, parts, true);
  return res;
}

// ---------------------------------------------------------------------------
// The paper's partition, emulated (section 3.2, Algorithm 1; section 4.2):
// every record is indexed by its HEALPix nested pixel at `order` and, in
// addition, by the pixels of the four positions shifted by +-R in RA and in
// Dec (R = the match radius in degrees, as Alg. 1 adds the error radius to
// the coordinates; RA shifts wrap around 360, Dec shifts stop at the poles).
// Records are compared only within a shared pixel; the decision is the exact
// one above, so the pairs missed are the partition's completeness loss.
// ---------------------------------------------------------------------------

// HEALPix nested pixel of (ra, dec) at Nside = 2^order, from the definitions
// of the HEALPix pixelisation (twelve base faces; equatorial zone |z| <= 2/3
// cut by two families of lines, polar caps by square-root scaled lines; the
// nested index interleaves the bits of the two in-face coordinates).
int64_t hp_nest(int order, double ra, double dec) {
  const int64_t ns = int64_t(1) << order;
  const double z = std::sin(dec * K64);
  const double za = std::fabs(z);
  double tt = ra / 90.0;  // phi / (pi/2), in [0, 4)
  tt = std::fmod(tt, 4.0);
  if (tt < 0) tt += 4.0;
  int64_t face, ix, iy;
  if (za <= 2.0 / 3.0) {
    const double t1 = ns * (0.5 + tt), t2 = ns * (z * 0.75);
    const int64_t jp = (int64_t)(t1 - t2), jm = (int64_t)(t1 + t2);
    const int64_t ifp = jp >> order, ifm = jm >> order;
    face = (ifp == ifm) ? (ifp | 4) : (ifp < ifm ? ifp : ifm + 8);
    ix = jm & (ns - 1);
    iy = ns - (jp & (ns - 1)) - 1;
  } else {
    int64_t ntt = (int64_t)tt;
    if (ntt > 3) ntt = 3;
    const double tp = tt - (double)ntt;
    // 1 - |z| = 2 sin^2(colatitude / 2), without cancellation
    const double sh = std::sin(0.5 * (90.0 - std::fabs(dec)) * K64);
    const double tmp = ns * std::sqrt(6.0) * sh;
    int64_t jp = (int64_t)(tp * tmp), jm = (int64_t)((1.0 - tp) * tmp);
    jp = std::min(jp, ns - 1);
    jm = std::min(jm, ns - 1);
    if (z >= 0) {
      face = ntt;
      ix = ns - jm - 1;
      iy = ns - jp - 1;
    } else {
      face = ntt + 8;
      ix = jp;
      iy = jm;
    }
  }
  int64_t ipf = 0;
  for (int b = 0; b < order; ++b) ipf |= ((ix >> b) & 1) << (2 * b) | ((iy >> b) & 1) << (2 * b + 1);
  return face * ns * ns + ipf;
}

// The distinct pixels of a record: its own and those of the four shifts.
int hp_quad(int order, double ra, double dec, double R, int64_t out[5]) {
  auto fold = [](double a) {
    a = std::fmod(a, 360.0);
    return a < 0 ? a + 360.0 : a;
  };
  int n = 0;
  auto put = [&](int64_t p) {
    for (int k = 0; k < n; ++k)
      if (out[k] == p) return;
    out[n++] = p;
  };
  put(hp_nest(order, ra, dec));
  put(hp_nest(order, fold(ra + R), dec));
  put(hp_nest(order, fold(ra - R), dec));
  put(hp_nest(order, ra, std::min(dec + R, 90.0)));
  put(hp_nest(order, ra, std::max(dec - R, -90.0)));
  return n;
}

// All m*n pairs, same decision. For small inputs only.
oracle_result* oracle_brute(const double* a_ra, const double* a_dec, int64_t na,
                            const double* b_ra, const double* b_dec, int64_t nb,
                            double r_arcsec, int nthreads, int* status) {
  *status = -1;
  if (na < 0 || nb < 0 || !(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return nullptr;
  int nt = resolve_threads(nthreads);
  omp_set_num_threads(nt);
  if (!check_inputs(a_ra, a_dec, na) || !check_inputs(b_ra, b_dec, nb)) return nullptr;
  auto* res = new oracle_result();
  *status = 0;
  Thresh t = make_thresh(r_arcsec);
  std::vector<std::vector<Hit>> parts(nt);
  std::vector<Stats> tst(nt);
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < na; ++i) {
      double cd = cos_dec64(a_dec[i]);
      for (int64_t j = 0; j < nb; ++j) {
        double sep;
        int o = decide(a_ra[i], a_dec[i], cd, b_ra[j], b_dec[j], cos_dec64(b_dec[j]), t, &sep);
        if (o == IN_QUAD || o == IN_TIE || o == OUT_QUAD) ++tst[tid].band;
        if (o == IN_TIE) ++tst[tid].ties;
        if (o == IN_FP64 || o == IN_QUAD || o == IN_TIE)
          parts[tid].push_back(Hit{(uint32_t)i, (uint32_t)j, sep});
      }
    }
  }
  for (auto& s : tst) {
    res->st.band += s.band;
    res->st.ties += s.ties;
  }
  res->st.candidates = na * nb;
  finish(res, parts, true);
  return res;
}

int64_t oracle_hp_nest(int order, double ra, double dec) {
  if (order < 0 || order > 13 || !valid_pos(ra, dec)) return -1;
  return hp_nest(order, ra, dec);
}

// Pairs the emulated paper partition finds (each once), exact decisions.
oracle_result* oracle_quad_direction(const double* a_ra, const double* a_dec, int64_t na,
                                     const double* b_ra, const double* b_dec, int64_t nb,
                                     double r_arcsec, int order, int nthreads, int* status) {
  *status = -1;
  if (na < 0 || nb < 0 || order < 0 || order > 13) return nullptr;
  if (!(r_arcsec > 0.0) || !(r_arcsec <= 3600.0)) return nullptr;
  int nt = resolve_threads(nthreads);
  omp_set_num_threads(nt);
  if (!check_inputs(a_ra, a_dec, na) || !check_inputs(b_ra, b_dec, nb)) return nullptr;
  auto* res = new oracle_result();
  *status = 0;
  const double R = r_arcsec / 3600.0;
  // (pixel, index) lists of B, sorted by pixel
  std::vector<std::pair<int64_t, uint32_t>> Bp;
  for (int64_t j = 0; j < nb; ++j) {
    int64_t px[5];
    int n = hp_quad(order, b_ra[j], b_dec[j], R, px);
    for (int k = 0; k < n; ++k) Bp.emplace_back(px[k], (uint32_t)j);
  }
  __gnu_parallel::sort(Bp.begin(), Bp.end());
  Thresh t = make_thresh(r_arcsec);
  std::vector<std::vector<Hit>> parts(nt);
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
#pragma omp for schedule(dynamic, 1024)
    for (int64_t i = 0; i < na; ++i) {
      int64_t pa[5];
      int n = hp_quad(order, a_ra[i], a_dec[i], R, pa);
      for (int k = 0; k < n; ++k) {
        auto it = std::lower_bound(Bp.begin(), Bp.end(), std::make_pair(pa[k], (uint32_t)0));
        for (; it != Bp.end() && it->first == pa[k]; ++it) {
          const uint32_t j = it->second;
          // count a pair once: in the smallest pixel the two records share
          int64_t pb[5];
          int m = hp_quad(order, b_ra[j], b_dec[j], R, pb);
          int64_t first = INT64_MAX;
          for (int u = 0; u < n; ++u)
            for (int v = 0; v < m; ++v)
              if (pa[u] == pb[v]) first = std::min(first, pa[u]);
          if (first != pa[k]) continue;
          double sep;
          int o = decide(a_ra[i], a_dec[i], cos_dec64(a_dec[i]), b_ra[j], b_dec[j], cos_dec64(b_dec[j]), t, &sep);
          if (o == IN_FP64 || o == IN_QUAD || o == IN_TIE) parts[tid].push_back(Hit{(uint32_t)i, j, sep});
        }
      }
    }
  }
  finish(res, parts, true);
  return res;
}

int64_t oracle_result_size(const oracle_result* r) { return (int64_t)r->hits.size(); }

void oracle_result_copy(const oracle_result* r, uint32_t* a, uint32_t* b, double* sep) {
  const size_t n = r->hits.size();
  for (size_t k = 0; k < n; ++k) {
    a[k] = r->hits[k].a;
    b[k] = r->hits[k].b;
    sep[k] = r->hits[k].sep;
  }
}

// candidates evaluated, pairs that needed binary128, true ties
void oracle_result_stats(const oracle_result* r, int64_t* out3) {
  out3[0] = r->st.candidates;
  out3[1] = r->st.band;
  out3[2] = r->st.ties;
}

void oracle_result_free(oracle_result* r) { delete r; }

}  // extern "C"
