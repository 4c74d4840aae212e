// batch.hip -- the batched form: thousands of independent cross-match jobs in
// one pass (the paper launches one kernel per calculation block, section
// 4.3.1; here every block of every job shares one partition, one sort and one
// persistent match launch).
//
// Each job gets a local frame computed on the device from its own sources:
// Dec zones start at the job's lowest Dec (minus r), RA bins span the job's
// own RA extent (or the full circle near a pole or when the extent is wide),
// and the zone height follows the job's density. Keys carry the job id in
// their top bits, (job << LB) | (zone << rb_j) | bin, so one global radix
// sort partitions every job at once and every B range stays inside its job.
//
// The FP32 filter of a job works on offsets from one snapped centre of the
// job's box (jobs are small cones, so the offsets are small); its threshold
// covers the FP32 rounding of offsets up to the box's extent E_j.
#include <hip/hip_runtime.h>

#include "hlc_kernels.hpp"

namespace hlc {

namespace {

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

constexpr int FT = 256;              // threads of the per-tile kernels (TI sources each)

__device__ inline double fold180(double x) {
  // x in (-360, 360] -> (-180, 180]
  if (x > 180.0) x -= 360.0;
  else if (x <= -180.0) x += 360.0;
  return x;
}

// Order-preserving encoding of a double as an unsigned 64-bit integer, so
// that atomicMin / atomicMax on the codes give the min / max of the values.
__device__ inline unsigned long long ord_enc(double d) {
  unsigned long long b = __double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double ord_dec(unsigned long long c) {
  return __longlong_as_double((c >> 63) ? (long long)(c & 0x7fffffffffffffffull) : (long long)~c);
}

__device__ inline double job_ref_ra(const BatchJob& J, const double* a_ra, const double* b_ra) {
  double ref = J.na > 0 ? a_ra[J.a_off] : (J.nb > 0 ? b_ra[J.b_off] : 0.0);
  return (ref >= 0.0 && ref <= 360.0) ? ref : 0.0;
}

// bounds[4 j + {0,1,2,3}] = codes of min Dec, max Dec, min and max RA offset
// from the job's reference RA (folded into (-180, 180])
__global__ void k_job_bounds_init(unsigned long long* bounds, int32_t njobs) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * njobs) return;
  bounds[i] = (i & 1) ? 0ull : ~0ull;  // min slots start high, max slots low
}

template <int TI>
__global__ __launch_bounds__(FT) void k_job_bounds(const BatchTile* __restrict__ tiles, uint32_t ntiles,
                                                   const BatchJob* __restrict__ jobs,
                                                   const double* __restrict__ a_ra,
                                                   const double* __restrict__ b_ra,
                                                   const double* __restrict__ ra,
                                                   const double* __restrict__ dec, int side_b,
                                                   unsigned long long* __restrict__ bounds, Counters* cnt) {
  if (blockIdx.x >= ntiles) return;
  const BatchTile T = tiles[blockIdx.x];
  // the tile's positions are in flight while the job's reference RA is read
  double av[TI], dv[TI];
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    const uint32_t k = j * FT + threadIdx.x;
    av[j] = 0.0;
    dv[j] = 0.0;
    if (k < T.count) {
      av[j] = ra[T.src + k];
      dv[j] = dec[T.src + k];
    }
  }
  const double ref = job_ref_ra(jobs[T.job], a_ra, b_ra);
  double dmin = 1e300, dmax = -1e300, omin = 1e300, omax = -1e300;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    if (j * FT + threadIdx.x >= T.count) continue;
    if (valid_pos(av[j], dv[j])) {
      dmin = fmin(dmin, dv[j]);
      dmax = fmax(dmax, dv[j]);
      const double o = fold180(av[j] - ref);
      omin = fmin(omin, o);
      omax = fmax(omax, o);
    } else {
      bad = true;
    }
  }
  if (bad) atomicOr(&cnt->err, side_b ? 2u : 1u);
  // wave, then block reductions: one atomic per block and bound
  for (int off = 32; off > 0; off >>= 1) {
    dmin = fmin(dmin, __shfl_xor(dmin, off));
    dmax = fmax(dmax, __shfl_xor(dmax, off));
    omin = fmin(omin, __shfl_xor(omin, off));
    omax = fmax(omax, __shfl_xor(omax, off));
  }
  __shared__ double s_b[FT / 64][4];
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_b[w][0] = dmin;
    s_b[w][1] = dmax;
    s_b[w][2] = omin;
    s_b[w][3] = omax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t u = 1; u < (blockDim.x + 63u) / 64u; ++u) {
      dmin = fmin(dmin, s_b[u][0]);
      dmax = fmax(dmax, s_b[u][1]);
      omin = fmin(omin, s_b[u][2]);
      omax = fmax(omax, s_b[u][3]);
    }
    if (dmin <= dmax) {
      unsigned long long* b = bounds + 4 * (size_t)T.job;
      atomicMin(&b[0], ord_enc(dmin));
      atomicMax(&b[1], ord_enc(dmax));
      atomicMin(&b[2], ord_enc(omin));
      atomicMax(&b[3], ord_enc(omax));
    }
  }
}

// One thread per job: the local frame from the job's bounds.
__global__ void k_job_frames(const BatchJob* __restrict__ jobs, int32_t njobs,
                             const double* __restrict__ a_ra, const double* __restrict__ b_ra,
                             const unsigned long long* __restrict__ bounds, int32_t lb_bits,
                             double h_factor, JobGeom* __restrict__ geo) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const BatchJob J = jobs[j];
  const double ref = job_ref_ra(J, a_ra, b_ra);
  double dmin = ord_dec(bounds[4 * j]), dmax = ord_dec(bounds[4 * j + 1]);
  double omin = ord_dec(bounds[4 * j + 2]), omax = ord_dec(bounds[4 * j + 3]);
  JobGeom G{};
  G.r_deg = J.r_arcsec / 3600.0;
  G.rpad_deg = G.r_deg * (1.0 + 1e-9) + 1e-12;
  if (!(dmin <= dmax)) {  // empty job
    dmin = dmax = 0.0;
    omin = omax = 0.0;
  }
  // RA frame: the job's folded RA extent, or the whole circle when the box is
  // wide or its padded Dec range comes near a pole
  const double span = omax - omin;
  const bool polar = dmax + 2.0 * G.rpad_deg >= 89.0 || dmin - 2.0 * G.rpad_deg <= -89.0;
  G.full_ra = (polar || span > 120.0) ? 1 : 0;
  if (G.full_ra) {
    G.ra0 = 0.0;
    G.ra_span = 360.0;
  } else {
    const double pad = 1e-7;
    G.ra0 = ref + omin - pad;
    if (G.ra0 < 0.0) G.ra0 += 360.0;
    if (G.ra0 >= 360.0) G.ra0 -= 360.0;
    G.ra_span = span + 2.0 * pad;
  }
  // zone height from the job's density: sqrt(GROUP / density), scaled
  const double dspan = fmax(dmax - dmin, 2.0 * G.rpad_deg);
  const double mid = 0.5 * (dmin + dmax);
  const double cmid = fmax(cos(mid * (M_PI / 180.0)), 1e-3);
  const double width = G.full_ra ? 360.0 * cmid : fmax(G.ra_span * cmid, 2.0 * G.rpad_deg);
  const double area_as2 = dspan * width * 3600.0 * 3600.0;
  const double n_mean = 0.5 * (double)(J.na + J.nb) + 1.0;
  double h = fmax(sqrt((double)GROUP * area_as2 / n_mean) * h_factor / 3600.0, 2.0001 * G.rpad_deg);
  G.d0 = fmax(dmin - 2.0 * G.rpad_deg, -90.0);
  const double dtop = fmin(dmax + 2.0 * G.rpad_deg, 90.0);
  int64_t nz = (int64_t)ceil((dtop - G.d0) / h) + 1;
  if (nz > (int64_t)J.zcap) {  // stay inside the job's table budget
    h = fmax((dtop - G.d0) / (double)(J.zcap - 1), 2.0001 * G.rpad_deg);
    nz = (int64_t)ceil((dtop - G.d0) / h) + 1;
    if (nz > (int64_t)J.zcap) nz = J.zcap;
  }
  G.h_deg = h;
  G.inv_h = 1.0 / h;
  G.nz = (int32_t)nz;
  int zb = 0;
  while ((1 << zb) < nz) ++zb;
  G.rb = lb_bits - zb;
  G.nbins = 1u << G.rb;
  G.bin_scale = (double)G.nbins / G.ra_span;
  G.zoff = J.zoff;
  // chord thresholds of the FP64 filter (same budget as the single call)
  const double r_rad = G.r_deg * (M_PI / 180.0);
  const double s = sin(0.5 * r_rad);
  const double U = 1.1102230246251565e-16, ETA = 4e-15;
  G.c_r = 2.0 * s;
  const double hi = G.c_r * (1.0 + 4.0 * U) + ETA;
  G.t_hi64 = hi * hi * (1.0 + 4.0 * U);
  const double lo = G.c_r * (1.0 - 4.0 * U) - ETA;
  G.t_lo64 = lo > 0 ? lo * lo * (1.0 - 4.0 * U) : -1.0;
  G.H_lo = J.H_lo;
  G.H_hi = J.H_hi;
  // FP32 frame: centre of the box (snapped to 2^-20) and E >= |u - c| there
  double cra, cdec, E;
  if (G.full_ra) {
    cra = 0.0;
    cdec = dmin > 0.0 ? 90.0 : (dmax < 0.0 ? -90.0 : 0.0);
    if (cdec == 0.0) {
      E = 2.0;
    } else {
      const double far = fmax(fabs(cdec - dmin), fabs(cdec - dmax)) + 2.0 * G.rpad_deg;
      E = fmin(2.0, far * (M_PI / 180.0) + 1e-6);
    }
  } else {
    cra = G.ra0 + 0.5 * G.ra_span;
    if (cra >= 360.0) cra -= 360.0;
    cdec = mid;
    E = fmin(2.0, (0.5 * dspan + 0.5 * G.ra_span + 4.0 * G.rpad_deg) * (M_PI / 180.0) + 1e-6);
  }
  double sd, cd, sa, ca;
  sincos_deg(cdec, &sd, &cd);
  sincos_deg(cra, &sa, &ca);
  G.cx = rint(cd * ca * 1048576.0) * (1.0 / 1048576.0);
  G.cy = rint(cd * sa * 1048576.0) * (1.0 / 1048576.0);
  G.cz = rint(sd * 1048576.0) * (1.0 / 1048576.0);
  E += 4.0 / 1048576.0;  // the snapped centre moves by <= sqrt(3) 2^-21
  const double v = 5.9604644775390625e-08;
  const double c = G.c_r * (1.0 + 4.0 * v) + 8.0 * v * E;
  const double T = c * c * (1.0 + 4.0 * v);
  float Tf = (float)T;
  if ((double)Tf < T) Tf = __uint_as_float(__float_as_uint(Tf) + 1u);
  G.thr32 = Tf;
  geo[j] = G;
}

__device__ inline int32_t job_zone(const JobGeom& G, double dec) {
  double t = floor((dec - G.d0) * G.inv_h);
  if (!(t >= 0.0)) return 0;
  if (t > (double)(G.nz - 1)) return G.nz - 1;
  return (int32_t)t;
}

__device__ inline uint32_t job_bin(const JobGeom& G, double ra) {
  double x = ra;
  if (!G.full_ra) {
    x = ra - G.ra0;
    if (x < 0.0) x += 360.0;
  }
  double t = floor(x * G.bin_scale);
  if (!(t >= 0.0)) return 0u;
  if (t > (double)(G.nbins - 1)) return G.nbins - 1;
  return (uint32_t)t;
}

// keys for one side; tiles never cross jobs (tile table built on the host).
// Entry positions are job-packed; values are the caller's global indices.
template <int TI>
__global__ __launch_bounds__(FT) void k_batch_keygen(const BatchTile* __restrict__ tiles,
                                                     uint32_t ntiles, const JobGeom* __restrict__ geo,
                                                     const double* __restrict__ ra,
                                                     const double* __restrict__ dec, int32_t lb_bits,
                                                     int halo, uint32_t n_total,
                                                     uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals, Counters* cnt) {
  if (blockIdx.x >= ntiles) return;
  const BatchTile T = tiles[blockIdx.x];
  double av[TI], dv[TI];
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    const uint32_t k = j * FT + threadIdx.x;
    av[j] = 0.0;
    dv[j] = 0.0;
    if (k < T.count) {
      av[j] = ra[T.src + k];
      dv[j] = dec[T.src + k];
    }
  }
  const JobGeom G = geo[T.job];
  const uint32_t jb = (uint32_t)T.job << lb_bits;
  uint32_t hkey[TI];
  uint64_t hm[TI];
  uint32_t wave_n = 0;
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    const uint32_t k = j * FT + threadIdx.x;
    const bool in = k < T.count;
    const bool ok = in && valid_pos(av[j], dv[j]);
    const double a = ok ? av[j] : 0.0, d = ok ? dv[j] : G.d0;
    const int32_t z = job_zone(G, d);
    const uint32_t b = job_bin(G, a);
    if (in) {
      keys[T.entry + k] = jb | ((uint32_t)z << G.rb) | b;
      vals[T.entry + k] = T.src + k;
    }
    hm[j] = 0;
    hkey[j] = 0;
    if (halo) {
      const int32_t zl = job_zone(G, d - G.rpad_deg), zh = job_zone(G, d + G.rpad_deg);
      const int32_t other = (zl != z) ? zl : zh;
      hkey[j] = jb | ((uint32_t)other << G.rb) | b;
      hm[j] = __ballot(ok && other != z);
      wave_n += (uint32_t)__popcll(hm[j]);
    }
  }
  if (!halo) return;
  // the block's halo copies placed with one atomic on the shared counter
  // (one per wave serialised every wave of the batch on one address)
  __shared__ uint32_t s_wc[FT / 64];
  __shared__ unsigned long long s_base[FT / 64];
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) s_wc[w] = wave_n;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (uint32_t u = 0; u < FT / 64; ++u) tot += s_wc[u];
    unsigned long long base = tot ? atomicAdd(&cnt->n_halo, tot) : 0ull;
    for (uint32_t u = 0; u < FT / 64; ++u) {
      s_base[u] = base;
      base += s_wc[u];
    }
  }
  __syncthreads();
  uint64_t pos = (uint64_t)n_total + s_base[w];
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    if ((hm[j] >> lane_id()) & 1ull) {
      keys[pos + rank_in(hm[j])] = hkey[j];
      vals[pos + rank_in(hm[j])] = (T.src + j * FT + threadIdx.x) | HALO_BIT;
    }
    pos += (uint64_t)__popcll(hm[j]);
  }
}

// FP32 records in the job frame, and FP64 (ra, dec) copies
__global__ __launch_bounds__(256) void k_batch_layout32(const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals, DevCount nc,
                                                        const double* __restrict__ ra,
                                                        const double* __restrict__ dec,
                                                        const JobGeom* __restrict__ geo, int32_t lb_bits,
                                                        Rec32* __restrict__ rec,
                                                        double2* __restrict__ radec) {
  // XCD-aware over the blocks the device-side count fills (the grid covers the
  // capacity): a job's sources, read in its sorted order, land in one L2
  const uint32_t n = nc.get(), nb = (n + blockDim.x - 1) / blockDim.x;
  if (blockIdx.x >= nb) return;
  const uint32_t p = xcd_block(blockIdx.x, nb) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t v = vals[p], i = v & IDX_MASK;
  const JobGeom& G = geo[keys[p] >> lb_bits];
  const double a = ra[i], d = dec[i];
  double sd, cd, sa, ca;
  sincos_deg(d, &sd, &cd);
  sincos_deg(a, &sa, &ca);
  Rec32 r;
  r.x = (float)(cd * ca - G.cx);
  r.y = (float)(cd * sa - G.cy);
  r.z = (float)(sd - G.cz);
  r.idx = v;
  rec[p] = r;
  radec[p] = make_double2(a, d);
}

// per-(job, zone) tables: RA margins and B zone starts; entry e of job j is
// zone e - zoff_j (zone nz_j: the end of the job's B entries)
__global__ __launch_bounds__(256) void k_batch_zone_tables(const JobGeom* __restrict__ geo,
                                                           int32_t njobs, const BatchJob* __restrict__ jobs,
                                                           uint32_t ztotal, int32_t lb_bits,
                                                           const uint32_t* __restrict__ keysB, DevCount nbc,
                                                           int32_t* __restrict__ zmarg,
                                                           uint32_t* __restrict__ zstart) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ztotal) return;
  int32_t lo = 0, hi = njobs - 1;  // last job with zoff <= e
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (jobs[mid].zoff <= e) lo = mid; else hi = mid - 1;
  }
  const int32_t j = lo;
  const JobGeom G = geo[j];
  const int32_t z = (int32_t)(e - jobs[j].zoff);
  if (z > G.nz) return;  // unused budget of this job
  const uint64_t K = ((uint64_t)j << lb_bits) + ((uint64_t)z << G.rb);
  const uint32_t nb = nbc.get();
  uint32_t l = 0, r = nb;
  if (K > 0xffffffffull) {
    l = nb;
  } else {
    while (l < r) {
      const uint32_t m = l + ((r - l) >> 1);
      if (keysB[m] < (uint32_t)K) l = m + 1; else r = m;
    }
  }
  zstart[e] = l;
  if (z == G.nz) return;
  const double zlo = G.d0 + (double)z * G.h_deg, zhi = zlo + G.h_deg;
  const double dstar = fmin(fmax(fabs(zlo), fabs(zhi)) + 1e-9, 90.0);
  int32_t m = -1;
  if (dstar + G.rpad_deg < 90.0) {
    double ss, cs, sd, cd;
    sincos_deg(G.rpad_deg, &ss, &cs);
    sincos_deg(dstar, &sd, &cd);
    const double x = ss / cd;
    if (x < 0.99) {
      const double delta = asin(x) * (180.0 / M_PI) * (1.0 + 1e-9) + 1e-12;
      const double mm = ceil(delta * G.bin_scale) + 2.0;
      if (2.0 * mm + 1.0 < (double)G.nbins) m = (int32_t)mm;
    }
  }
  zmarg[e] = m;  // -1: the whole zone of the job
}

__device__ inline uint32_t gallop_lower_b(const uint32_t* keys, uint32_t K, uint32_t hint, uint32_t lo,
                                          uint32_t hi) {
  if (hint < lo) hint = lo;
  if (hint > hi) hint = hi;
  int64_t l, r;
  if (hint < hi && keys[hint] < K) {
    int64_t a = hint, step = 1, b = a + 1;
    while (b < (int64_t)hi && keys[b] < K) {
      a = b;
      step <<= 1;
      b = a + step;
    }
    if (b > (int64_t)hi) b = hi;
    l = a + 1;
    r = b;
  } else {
    int64_t b = hint, step = 1, a = b - 1;
    while (a >= (int64_t)lo && keys[a] >= K) {
      b = a;
      step <<= 1;
      a = b - step;
    }
    l = a < (int64_t)lo ? (int64_t)lo : a + 1;
    r = b;
  }
  while (l < r) {
    int64_t mid = (l + r) >> 1;
    if (keys[mid] >= K) r = mid; else l = mid + 1;
  }
  return (uint32_t)l;
}
__device__ inline uint32_t gallop_upper_b(const uint32_t* keys, uint32_t K, uint32_t hint, uint32_t lo,
                                          uint32_t hi) {
  if (K == 0xffffffffu) return hi;
  return gallop_lower_b(keys, K + 1u, hint, lo, hi);
}

// per group of 16 A entries: B ranges (runs split by job and zone)
__global__ __launch_bounds__(256) void k_batch_ranges(const uint32_t* __restrict__ keysA, DevCount nac,
                                                      const uint32_t* __restrict__ lb,
                                                      const uint32_t* __restrict__ keysB,
                                                      const JobGeom* __restrict__ geo, int32_t lb_bits,
                                                      const int32_t* __restrict__ zmarg,
                                                      const uint32_t* __restrict__ zstart,
                                                      GroupRanges* __restrict__ out,
                                                      uint32_t* __restrict__ cost_key,
                                                      uint32_t* __restrict__ cost_val) {
  const uint32_t na = nac.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  const uint32_t grp = blockIdx.x * blockDim.x + threadIdx.x;
  if (grp >= (nac.cap + GROUP - 1) / GROUP) return;
  if (grp >= ngroups) {  // padding of the LPT order: sorts last, never processed
    cost_key[grp] = 0xffffffffu;
    cost_val[grp] = grp;
    return;
  }
  const uint32_t p0 = grp * GROUP;
  const uint32_t cnt = min((uint32_t)GROUP, na - p0);
  RangeList L;
  L.clear();
  auto add = [&](uint32_t a, uint32_t b) { L.add(a, b); };
  uint32_t q = 0;
  while (q < cnt) {
    const uint32_t k0 = keysA[p0 + q];
    const int32_t j = (int32_t)(k0 >> lb_bits);
    const JobGeom G = geo[j];
    const uint32_t zkey = k0 >> G.rb;  // (job, zone)
    uint32_t qe = q;
    while (qe + 1 < cnt && (keysA[p0 + qe + 1] >> G.rb) == zkey && (keysA[p0 + qe + 1] >> lb_bits) == (uint32_t)j)
      ++qe;
    const int32_t z = (int32_t)(zkey & ((1u << (lb_bits - G.rb)) - 1u));
    const uint32_t zs = zstart[G.zoff + z], ze = zstart[G.zoff + z + 1];
    const int64_t nbins = G.nbins;
    const int64_t bf = k0 & (G.nbins - 1), bl = keysA[p0 + qe] & (G.nbins - 1);
    const int32_t m = zmarg[G.zoff + z];
    const int64_t lo = bf - m, hi = bl + m;
    const uint32_t jz = (uint32_t)j << lb_bits | ((uint32_t)z << G.rb);
    if (zs < ze) {
      if (m < 0 || hi - lo + 1 >= nbins) {
        add(zs, ze);
      } else if (!G.full_ra) {
        uint32_t s = gallop_lower_b(keysB, jz | (uint32_t)(lo < 0 ? 0 : lo), lb[p0 + q], zs, ze);
        uint32_t e = gallop_upper_b(keysB, jz | (uint32_t)(hi > nbins - 1 ? nbins - 1 : hi), lb[p0 + qe],
                                    zs, ze);
        add(s, e);
      } else {
        uint32_t s = gallop_lower_b(keysB, jz | (uint32_t)(lo < 0 ? 0 : lo), lb[p0 + q], zs, ze);
        uint32_t e = gallop_upper_b(keysB, jz | (uint32_t)(hi > nbins - 1 ? nbins - 1 : hi), lb[p0 + qe],
                                    zs, ze);
        if (hi > nbins - 1) add(zs, gallop_upper_b(keysB, jz | (uint32_t)(hi - nbins), zs, zs, ze));
        add(s, e);
        if (lo < 0) add(gallop_lower_b(keysB, jz | (uint32_t)(nbins + lo), ze, zs, ze), ze);
      }
    }
    q = qe + 1;
  }
  GroupRanges R;
  uint32_t work = 0;
  const int n = L.n;
#pragma unroll
  for (int t = 0; t < MAXR; ++t) {
    R.start[t] = t < n ? L.s[t] : 0u;
    R.end[t] = t < n ? L.e[t] : 0u;
    if (t < n) work += L.e[t] - L.s[t];
  }
  R.count = (uint32_t)n;
  R.pad_[0] = R.pad_[1] = R.pad_[2] = 0u;
  out[grp] = R;
  // LPT order: most B work first (ascending sort of the complement)
  cost_key[grp] = 0xfffffffeu - min(work + 1u, 0xfffffffeu);
  cost_val[grp] = grp;
}

// ---------------------------------------------------------------------------
// persistent match kernel over LPT-ordered groups
// ---------------------------------------------------------------------------
constexpr int MT = 256;
constexpr int WAVES = MT / 64;
constexpr int QCAP = 64 * (GROUP + 1);

__device__ inline void bemit(bool in, uint32_t ia, uint32_t ib, double sep, int32_t job,
                             const OutArgs& o, unsigned long long* job_count) {
  emit_wave(in, ia, ib, sep, o);
  if (!job_count) return;
  // one atomic per distinct job among the wave's pairs (the four groups of
  // a wave seldom span more than two jobs)
  uint64_t rem = __ballot(in);
  while (rem) {
    const uint32_t leader = (uint32_t)__builtin_ctzll(rem);
    const int32_t j0 = __shfl(job, (int)leader);
    const uint64_t same = __ballot(in && job == j0);
    if (lane_id() == leader) atomicAdd(&job_count[j0], (unsigned long long)__popcll(same));
    rem &= ~same;
  }
}

__device__ inline void bband(bool band, uint32_t ia, uint32_t ib, int32_t job, const OutArgs& o) {
  uint64_t m = __ballot(band);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(&o.cnt->n_band, (unsigned long long)__popcll(m));
  base = __shfl(base, (int)leader);
  if (band) {
    unsigned long long slot = base + rank_in(m);
    if (slot < o.band_cap) {
      o.band[slot] = make_uint2(ia, ib);
      o.band_job[slot] = (uint32_t)job;
    }
  }
}

template <bool FP32>
__device__ void bflush(const BatchMatchArgs& a, const OutArgs& o, const uint2* q, uint32_t qn) {
  const uint32_t lane = lane_id();
  count_candidates(qn, o);
  for (uint32_t b0 = 0; b0 < qn; b0 += 64) {
    const uint32_t e = b0 + lane;
    bool in = false, band = false;
    uint32_t ia = 0, ib = 0;
    int32_t job = 0;
    double sep = 0.0;
    if (e < qn) {
      const uint2 ent = q[e];
      const uint32_t kA = a.keysA[ent.x], kB = a.keysB[ent.y];
      job = (int32_t)(kA >> a.lb_bits);
      const JobGeom& G = a.geo[job];
      const bool same = (kA >> G.rb) == (kB >> G.rb);  // same job and zone
      if (FP32) {
        const double2 pa = a.radecA[ent.x], pb = a.radecB[ent.y];
        ia = a.recA32[ent.x].idx & IDX_MASK;
        ib = a.recB32[ent.y].idx & IDX_MASK;
        const double h = haversine64(pa.x, pa.y, pb.x, pb.y);
        in = same && h < G.H_lo;
        band = same && !in && h <= G.H_hi;
        if (in) sep = 2.0 * asin(sqrt(h)) * RAD2ARCSEC;
      } else {
        const Rec64 A = a.recA64[ent.x], B = a.recB64[ent.y];
        const double dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
        const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
        ia = A.idx & IDX_MASK;
        ib = B.idx & IDX_MASK;
        in = same && d2 <= G.t_lo64;
        band = same && !in && d2 <= G.t_hi64;
        if (in) sep = 2.0 * asin(0.5 * sqrt(d2)) * RAD2ARCSEC;
      }
    }
    bemit(in, ia, ib, sep, job, o, a.job_count);
    bband(band, ia, ib, job, o);
  }
}

template <bool FP32, int N>
__device__ inline void bsteps(float ax32, float ay32, float az32, double ax, double ay, double az,
                              bool a_ok, float bx32, float by32, float bz32, double bx, double by,
                              double bz, float thr32, double thr64, uint32_t a_pos, uint32_t b_pos0,
                              uint2* q, uint32_t& qn) {
  bool hit;
  if (FP32) {
    const float dx = ax32 - row_bcast<N>(bx32), dy = ay32 - row_bcast<N>(by32), dz = az32 - row_bcast<N>(bz32);
    hit = a_ok && fmaf(dx, dx, fmaf(dy, dy, dz * dz)) <= thr32;
  } else {
    const double dx = ax - row_bcast<N>(bx), dy = ay - row_bcast<N>(by), dz = az - row_bcast<N>(bz);
    hit = a_ok && fma(dx, dx, fma(dy, dy, dz * dz)) <= thr64;
  }
  const uint64_t m = __ballot(hit);
  if (m) {
    if (hit) q[qn + rank_in(m)] = make_uint2(a_pos, b_pos0 + N);
    qn += (uint32_t)__popcll(m);
  }
  if constexpr (N + 1 < GROUP)
    bsteps<FP32, N + 1>(ax32, ay32, az32, ax, ay, az, a_ok, bx32, by32, bz32, bx, by, bz, thr32, thr64,
                        a_pos, b_pos0, q, qn);
}

template <bool FP32>
__global__ __launch_bounds__(MT) void k_batch_match(BatchMatchArgs a, OutArgs o) {
  __shared__ uint2 s_q[WAVES][QCAP];
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t row = lane >> 4, l16 = lane & 15u;
  uint2* q = s_q[w];
  uint32_t qn = 0;
  const uint32_t na = a.na.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  // persistent: wave w of W takes the four groups at LPT positions
  // 4 (w + i W), i = 0, 1, ... (largest first, dealt round-robin; no queue
  // atomics); every wave leaves after its last item
  const uint32_t W = gridDim.x * WAVES;
  const uint32_t wid = blockIdx.x * WAVES + w;
  for (uint32_t item = 4u * wid; item < ngroups; item += 4u * W) {
    const uint32_t slot = item + row;
    const bool grp_ok = slot < ngroups;
    const uint32_t grp = grp_ok ? a.order[slot] : 0u;
    const GroupRanges* R = grp_ok ? a.ranges + grp : nullptr;
    const uint32_t a_pos = grp * GROUP + l16;
    bool a_ok = grp_ok && a_pos < na;
    float ax32 = 0.f, ay32 = 0.f, az32 = 0.f, thr32 = 0.f;
    double ax = 0.0, ay = 0.0, az = 0.0, thr64 = 0.0;
    if (a_ok) {
      const JobGeom& G = a.geo[a.keysA[a_pos] >> a.lb_bits];
      if (FP32) {
        const Rec32 A = a.recA32[a_pos];
        ax32 = A.x; ay32 = A.y; az32 = A.z;
        thr32 = G.thr32;
      } else {
        const Rec64 A = a.recA64[a_pos];
        ax = A.x; ay = A.y; az = A.z;
        thr64 = G.t_hi64;
      }
    }
    uint32_t ri = 0, pos = 0, end = 0;
    bool active = false;
    auto seek = [&]() {
      active = false;
      if (R == nullptr) return;
      const uint32_t n = R->count;
      while (ri < n) {
        pos = R->start[ri];
        end = R->end[ri];
        if (pos < end) { active = true; return; }
        ++ri;
      }
    };
    seek();
    while (__ballot(active)) {
      float bx32 = 1e30f, by32 = 1e30f, bz32 = 1e30f;
      double bx = 1e30, by = 1e30, bz = 1e30;
      const uint32_t b0 = pos;
      if (active && pos + l16 < end) {
        if (FP32) {
          const Rec32 B = a.recB32[pos + l16];
          bx32 = B.x; by32 = B.y; bz32 = B.z;
        } else {
          const Rec64 B = a.recB64[pos + l16];
          bx = B.x; by = B.y; bz = B.z;
        }
      }
      bsteps<FP32, 0>(ax32, ay32, az32, ax, ay, az, a_ok && active, bx32, by32, bz32, bx, by, bz, thr32,
                      thr64, a_pos, b0, q, qn);
      if (active) {
        pos += GROUP;
        if (pos >= end) {
          ++ri;
          seek();
        }
      }
      if (qn >= 64) {
        bflush<FP32>(a, o, q, qn);
        qn = 0;
      }
    }
  }
  if (qn) bflush<FP32>(a, o, q, qn);
}

// band list of the batch (each entry carries its job)
__global__ __launch_bounds__(256) void k_batch_certify(const double* __restrict__ a_ra,
                                                       const double* __restrict__ a_dec,
                                                       const double* __restrict__ b_ra,
                                                       const double* __restrict__ b_dec,
                                                       const BatchJob* __restrict__ jobs, OutArgs o,
                                                       unsigned long long* job_count) {
  unsigned long long n = o.cnt->n_band;
  if (n > o.band_cap) n = o.band_cap;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint2 e = o.band[i];
    const uint32_t j = o.band_job[i];
    const BatchJob J = jobs[j];
    const double ra1 = a_ra[e.x], de1 = a_dec[e.x], ra2 = b_ra[e.y], de2 = b_dec[e.y];
    const double h = haversine64(ra1, de1, ra2, de2);
    bool in = false;
    double sep = 0.0;
    if (h < J.H_lo) {
      in = true;
      sep = 2.0 * asin(sqrt(h)) * RAD2ARCSEC;
    } else if (h <= J.H_hi) {
      const dd hd = haversine_dd(ra1, de1, ra2, de2);
      const dd Hd = threshold_dd(J.r_arcsec);
      const dd diff = dd_add(hd, dd_neg(Hd));
      atomicAdd(&o.cnt->n_ties, 1ull);
      if (diff.hi <= TIE_REL * Hd.hi) {
        in = true;
        sep = 2.0 * asin(sqrt(hd.hi)) * RAD2ARCSEC;
      }
    }
    if (in) {
      emit_one(e.x, e.y, sep, o);
      if (job_count) atomicAdd(&job_count[j], 1ull);
    }
  }
}

__global__ void k_zero_u64(unsigned long long* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

}  // namespace

void launch_job_bounds_init(unsigned long long* bounds, int32_t njobs, hipStream_t s) {
  k_job_bounds_init<<<cdiv(4 * (uint64_t)njobs, 256), 256, 0, s>>>(bounds, njobs);
}

void launch_job_bounds(const BatchTile* tiles, uint32_t ntiles, int tile, const BatchJob* jobs,
                       const double* a_ra, const double* b_ra, const double* ra, const double* dec, bool side_b,
                       unsigned long long* bounds, Counters* cnt, hipStream_t s) {
  if (ntiles == 0) return;
  const int sb = side_b ? 1 : 0;
#define HLC_JOB_BOUNDS(TI) \
  k_job_bounds<TI><<<ntiles, FT, 0, s>>>(tiles, ntiles, jobs, a_ra, b_ra, ra, dec, sb, bounds, cnt)
  switch (tile) {
    case 256: HLC_JOB_BOUNDS(1); break;
    case 512: HLC_JOB_BOUNDS(2); break;
    case 2048: HLC_JOB_BOUNDS(8); break;
    default: HLC_JOB_BOUNDS(4); break;
  }
#undef HLC_JOB_BOUNDS
}

void launch_job_frames(const BatchJob* jobs, int32_t njobs, const double* a_ra, const double* b_ra,
                       const unsigned long long* bounds, int32_t lb_bits, double h_factor, JobGeom* geo,
                       hipStream_t s) {
  k_job_frames<<<cdiv(njobs, 256), 256, 0, s>>>(jobs, njobs, a_ra, b_ra, bounds, lb_bits, h_factor, geo);
}

void launch_batch_keygen(const BatchTile* tiles, uint32_t ntiles, int tile, const JobGeom* geo, const double* ra,
                         const double* dec, int32_t lb_bits, bool halo, uint32_t n_total, uint32_t* keys,
                         uint32_t* vals, Counters* cnt, hipStream_t s) {
  if (ntiles == 0) return;
  const int h = halo ? 1 : 0;
#define HLC_BATCH_KEYGEN(TI) \
  k_batch_keygen<TI><<<ntiles, FT, 0, s>>>(tiles, ntiles, geo, ra, dec, lb_bits, h, n_total, keys, vals, cnt)
  switch (tile) {
    case 256: HLC_BATCH_KEYGEN(1); break;
    case 512: HLC_BATCH_KEYGEN(2); break;
    case 2048: HLC_BATCH_KEYGEN(8); break;
    default: HLC_BATCH_KEYGEN(4); break;
  }
#undef HLC_BATCH_KEYGEN
}

void launch_batch_layout32(const uint32_t* keys, const uint32_t* vals, const DevCount& n, const double* ra,
                           const double* dec, const JobGeom* geo, int32_t lb_bits, Rec32* rec,
                           double2* radec, hipStream_t s) {
  if (n.cap == 0) return;
  k_batch_layout32<<<cdiv(n.cap, 256), 256, 0, s>>>(keys, vals, n, ra, dec, geo, lb_bits, rec, radec);
}

void launch_batch_zone_tables(const JobGeom* geo, int32_t njobs, const BatchJob* jobs, uint32_t ztotal,
                              int32_t lb_bits, const uint32_t* keysB, const DevCount& nb, int32_t* zmarg,
                              uint32_t* zstart, hipStream_t s) {
  k_batch_zone_tables<<<cdiv(ztotal, 256), 256, 0, s>>>(geo, njobs, jobs, ztotal, lb_bits, keysB, nb, zmarg,
                                                        zstart);
}

void launch_batch_ranges(const uint32_t* keysA, const DevCount& na, const uint32_t* lb, const uint32_t* keysB,
                         const JobGeom* geo, int32_t lb_bits, const int32_t* zmarg, const uint32_t* zstart,
                         GroupRanges* out, uint32_t* cost_key, uint32_t* cost_val, hipStream_t s) {
  uint32_t ng = cdiv(na.cap, GROUP);
  if (ng == 0) return;
  k_batch_ranges<<<cdiv(ng, 256), 256, 0, s>>>(keysA, na, lb, keysB, geo, lb_bits, zmarg, zstart, out,
                                               cost_key, cost_val);
}

void launch_batch_match(const BatchMatchArgs& a, const OutArgs& o, bool fp32, uint32_t nblocks,
                        hipStream_t s) {
  if (fp32) k_batch_match<true><<<nblocks, MT, 0, s>>>(a, o);
  else k_batch_match<false><<<nblocks, MT, 0, s>>>(a, o);
}

void launch_batch_certify(const double* a_ra, const double* a_dec, const double* b_ra, const double* b_dec,
                          const BatchJob* jobs, const OutArgs& o, unsigned long long* job_count,
                          hipStream_t s) {
  k_batch_certify<<<256, 256, 0, s>>>(a_ra, a_dec, b_ra, b_dec, jobs, o, job_count);
}

void launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t s) {
  if (n == 0) return;
  k_zero_u64<<<std::min<uint32_t>(cdiv(n, 256), 1024), 256, 0, s>>>(p, n);
}

}  // namespace hlc
