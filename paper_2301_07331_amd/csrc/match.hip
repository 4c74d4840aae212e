// match.hip -- the distance kernels of the cross-match (the paper's kernel
// module, sections 3.1 and 4.3.1), redesigned for CDNA4 wave64.
//
// Work unit: a group of 16 consecutive A sources in (zone, RA-bin) order, one
// source per lane of a 16-lane DPP row; a wave holds four groups. Each group
// scans at most MAXR contiguous ranges of the sorted B arrays (its Dec zone,
// RA window split at the seam, whole ring near a pole). Sixteen B records at a
// time are loaded, one per lane, and broadcast across the row with DPP
// row_newbcast, so every lane compares its A with every B without LDS traffic.
//
// Filters (both end in the same exact decision):
//   FP64: chord^2 = |u_a - u_b|^2 of FP64 unit vectors. Candidates are pairs
//     with chord^2 <= t_hi64; below t_lo64 the pair is certainly in and its
//     separation is 2 asin(chord/2). Between the two it goes to the band list.
//   FP32: offsets from FP32 cell centres, moved to the frame of the group's
//     first cell (centre differences are exact in FP32), compared against a
//     per-group bound that covers the FP32 rounding; every candidate is then
//     certified with the FP64 haversine of its (ra, dec), and only those within
//     the FP64 band of r go to the band list.
// The paper writes a dense "1" matrix per calculation block (section 4.3.2);
// here hits are compacted per wave (ballot + mbcnt rank) into an LDS queue,
// certified with all 64 lanes busy, and written with one atomic per wave.
//
// FP64 chord error budget (u = 2^-53): each unit-vector component is a
// product of two degree-reduced sin/cos values (each within ~1.5 ulp) and has
// an absolute error <= 4u; a chord component then errs by <= 8u + u|d|, so
// |chord_fp64 - chord| <= sqrt(3)*8u + u*chord ~= 1.6e-15. ETA64 = 4e-15 is
// used for the thresholds (2.5x margin for the device libm).
//
// FP32 filter budget (v = 2^-24): with E >= |u - c0| for every source of the
// group's window, a shifted offset errs by <= 2vE per component, a difference
// by <= 4vE + v|d|, so chord_fp32 <= chord(1 + v) + sqrt(3)*4vE and the group
// threshold (c_r(1+4v) + 8vE)^2 (1+4v) never rejects a true pair.
#include <hip/hip_runtime.h>

#include "hlc_kernels.hpp"

namespace hlc {

namespace {

constexpr int MT = 256;                 // threads per block
constexpr int WAVES = MT / 64;
constexpr int QCAP = 64 * (GROUP + 1);  // per-wave queue (flushed after each 16-step batch)

__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
  // consecutive logical blocks on the same XCD (dispatch is round-robin over 8)
  uint32_t q = nblocks >> 3, r = nblocks & 7u, x = bid & 7u, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// Thresholds of the eq. (4) radius of one pair (arcsec): chord^2 bounds of
// the FP64 filter and the haversine band. r carries <= 3u from the sqrt and
// products and the degree sine <= 3u, so 32u margins hold.
__device__ inline double pair_radius(const MatchArgs& a, uint32_t ia, uint32_t ib) {
  const double ea = a.a_err[ia], eb = a.b_err[ib];
  return a.k_sigma * sqrt(ea * ea + eb * eb);
}
__device__ inline void pair_chord_thr(double r_as, double& tlo, double& thi) {
  double s, c;
  sincos_deg(0.5 * r_as * (1.0 / 3600.0), &s, &c);
  const double U = 1.1102230246251565e-16, ETA = 4e-15;
  const double cr = 2.0 * s;
  const double hi = cr * (1.0 + 32.0 * U) + ETA;
  thi = hi * hi * (1.0 + 32.0 * U);
  const double lo = cr * (1.0 - 32.0 * U) - ETA;
  tlo = lo > 0 ? lo * lo * (1.0 - 32.0 * U) : -1.0;
}
__device__ inline void pair_hav_thr(double r_as, double& Hlo, double& Hhi) {
  double s, c;
  sincos_deg(0.5 * r_as * (1.0 / 3600.0), &s, &c);
  const double H = s * s;
  Hlo = H * (1.0 - EPS_BAND);
  Hhi = H * (1.0 + EPS_BAND);
}

__device__ inline void emit_band(bool band, uint32_t ia, uint32_t ib, const OutArgs& o) {
  uint64_t m = __ballot(band);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(&o.cnt->n_band, (unsigned long long)__popcll(m));
  base = __shfl(base, (int)leader);
  if (band) {
    unsigned long long slot = base + rank_in(m);
    if (slot < o.band_cap) o.band[slot] = make_uint2(ia, ib);
  }
}

// ---------------------------------------------------------------------------
// FP64 form
// ---------------------------------------------------------------------------
__device__ inline void flush64(const MatchArgs& a, const OutArgs& o, const uint2* q, uint32_t qn) {
  const uint32_t lane = lane_id();
  count_candidates(qn, o);
  for (uint32_t b0 = 0; b0 < qn; b0 += 64) {
    const uint32_t e = b0 + lane;
    bool in = false, band = false;
    uint32_t ia = 0, ib = 0;
    double sep = 0.0;
    if (e < qn) {
      uint2 ent = q[e];
      Rec64 A = a.recA64[ent.x];
      Rec64 B = a.recB64[ent.y];
      double dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
      double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
      ia = A.idx & IDX_MASK;
      ib = B.idx & IDX_MASK;
      // a group straddling two zones also scans the other zone, whose B
      // entries include halo copies of B sources this A meets in its own
      // zone: only entries of the A source's own zone count
      const bool same_zone = ((a.keysA[ent.x] ^ a.keysB[ent.y]) >> a.geom.rb) == 0u;
      bool keep = same_zone && (!a.self_only || ia < ib);
      if (keep && a.hp_order >= 0) {
        // paper-scheme emulation: count the pair in the smallest shared pixel
        uint32_t pa[5], pb[5];
        const double2 ca = a.radecA[ent.x], cb = a.radecB[ent.y];
        const int na_ = hp_quad(a.hp_order, ca.x, ca.y, a.hp_R, pa);
        const int nb_ = hp_quad(a.hp_order, cb.x, cb.y, a.hp_R, pb);
        uint32_t first = 0xffffffffu;
        for (int u = 0; u < na_; ++u)
          for (int v = 0; v < nb_; ++v)
            if (pa[u] == pb[v] && pa[u] < first) first = pa[u];
        keep = first == a.keysA[ent.x];
      }
      double tlo = a.t_lo64, thi = a.t_hi64;
      if (a.a_err) pair_chord_thr(pair_radius(a, ia, ib), tlo, thi);
      in = keep && d2 <= tlo;
      band = keep && !in && d2 <= thi;
      if (in) sep = 2.0 * asin(0.5 * sqrt(d2)) * RAD2ARCSEC;
    }
    emit_wave(in, ia, ib, sep, o);
    emit_band(band, ia, ib, o);
  }
}

template <int N>
__device__ inline void step64(double ax, double ay, double az, bool a_ok, const double3& b,
                              double thr, uint32_t a_pos, uint32_t b_pos0, uint2* q, uint32_t& qn) {
  const double bx = row_bcast<N>(b.x), by = row_bcast<N>(b.y), bz = row_bcast<N>(b.z);
  const double dx = ax - bx, dy = ay - by, dz = az - bz;
  const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const bool hit = a_ok && d2 <= thr;
  const uint64_t m = __ballot(hit);
  if (m) {
    if (hit) q[qn + rank_in(m)] = make_uint2(a_pos, b_pos0 + N);
    qn += (uint32_t)__popcll(m);
  }
}

template <int N>
__device__ inline void steps64(double ax, double ay, double az, bool a_ok, const double3& b,
                               double thr, uint32_t a_pos, uint32_t b_pos0, uint2* q, uint32_t& qn) {
  step64<N>(ax, ay, az, a_ok, b, thr, a_pos, b_pos0, q, qn);
  if constexpr (N + 1 < GROUP) steps64<N + 1>(ax, ay, az, a_ok, b, thr, a_pos, b_pos0, q, qn);
}

// Per-row cursor over up to MAXR ranges (read from global memory: the
// range table is indexed dynamically and must not live in registers).
struct Cursor {
  uint32_t ri, pos, end;
  bool active;
};

__device__ inline void cursor_seek(Cursor& c, const GroupRanges* R) {
  c.active = false;
  if (R == nullptr) return;
  const uint32_t n = R->count;
  while (c.ri < n) {
    c.pos = R->start[c.ri];
    c.end = R->end[c.ri];
    if (c.pos < c.end) { c.active = true; return; }
    ++c.ri;
  }
}

__device__ inline void cursor_advance(Cursor& c, const GroupRanges* R) {
  c.pos += GROUP;
  if (c.pos < c.end) return;
  ++c.ri;
  cursor_seek(c, R);
}

__global__ __launch_bounds__(MT) void k_match64(MatchArgs a, OutArgs o) {
  __shared__ uint2 s_q[WAVES][QCAP];
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t row = lane >> 4, l16 = lane & 15u;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t grp = (blk * WAVES + w) * 4u + row;
  uint2* q = s_q[w];
  uint32_t qn = 0;

  const uint32_t na = a.na.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  const bool grp_ok = grp < ngroups;
  const GroupRanges* R = grp_ok ? a.ranges + grp : nullptr;
  const uint32_t a_pos = grp * GROUP + l16;
  bool a_ok = grp_ok && a_pos < na;
  double ax = 0.0, ay = 0.0, az = 0.0;
  if (a_ok) {
    Rec64 A = a.recA64[a_pos];
    ax = A.x; ay = A.y; az = A.z;
    if (a.skip_halo_a && (A.idx & HALO_BIT)) a_ok = false;
  }
  const double thr = a.t_hi64;
  Cursor c;
  c.ri = 0;
  cursor_seek(c, R);
  while (__ballot(c.active)) {
    double3 b = make_double3(1e30, 1e30, 1e30);
    uint32_t b0 = c.pos;
    if (c.active && c.pos + l16 < c.end) {
      Rec64 B = a.recB64[c.pos + l16];
      b = make_double3(B.x, B.y, B.z);
    }
    steps64<0>(ax, ay, az, a_ok && c.active, b, thr, a_pos, b0, q, qn);
    if (c.active) cursor_advance(c, R);
    if (qn >= 64) {
      flush64(a, o, q, qn);
      qn = 0;
    }
  }
  if (qn) flush64(a, o, q, qn);
}

// ---------------------------------------------------------------------------
// FP32 form
// ---------------------------------------------------------------------------
__device__ inline void cell_centre(const MatchArgs& a, uint32_t k, double& cx, double& cy, double& cz) {
  const Geom& g = a.geom;
  double2 zc = a.zone_cs[key_zone(g, k)];
  double2 sc = a.super_cs[key_bin(g, k) >> g.cell_shift];
  cx = rint(zc.x * sc.x * 1048576.0) * (1.0 / 1048576.0);
  cy = rint(zc.x * sc.y * 1048576.0) * (1.0 / 1048576.0);
  cz = rint(zc.y * 1048576.0) * (1.0 / 1048576.0);
}

__device__ inline void flush32(const MatchArgs& a, const OutArgs& o, const uint2* q, uint32_t qn) {
  const uint32_t lane = lane_id();
  count_candidates(qn, o);
  for (uint32_t b0 = 0; b0 < qn; b0 += 64) {
    const uint32_t e = b0 + lane;
    bool in = false, band = false;
    uint32_t ia = 0, ib = 0;
    double sep = 0.0;
    if (e < qn) {
      uint2 ent = q[e];
      double2 pa = a.radecA[ent.x];
      double2 pb = a.radecB[ent.y];
      ia = a.recA32[ent.x].idx & IDX_MASK;
      ib = a.recB32[ent.y].idx & IDX_MASK;
      double h = haversine64(pa.x, pa.y, pb.x, pb.y);
      const bool same_zone = ((a.keysA[ent.x] ^ a.keysB[ent.y]) >> a.geom.rb) == 0u;
      const bool keep = same_zone && (!a.self_only || ia < ib);
      double Hlo = a.H_lo, Hhi = a.H_hi;
      if (a.a_err) pair_hav_thr(pair_radius(a, ia, ib), Hlo, Hhi);
      in = keep && h < Hlo;
      band = keep && !in && h <= Hhi;
      if (in) sep = 2.0 * asin(sqrt(h)) * RAD2ARCSEC;
    }
    emit_wave(in, ia, ib, sep, o);
    emit_band(band, ia, ib, o);
  }
}

template <int N>
__device__ inline void steps32(float ax, float ay, float az, bool a_ok, const float3& b, float thr,
                               uint32_t a_pos, uint32_t b_pos0, uint2* q, uint32_t& qn) {
  const float bx = row_bcast<N>(b.x), by = row_bcast<N>(b.y), bz = row_bcast<N>(b.z);
  const float dx = ax - bx, dy = ay - by, dz = az - bz;
  const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const bool hit = a_ok && d2 <= thr;
  const uint64_t m = __ballot(hit);
  if (m) {
    if (hit) q[qn + rank_in(m)] = make_uint2(a_pos, b_pos0 + N);
    qn += (uint32_t)__popcll(m);
  }
  if constexpr (N + 1 < GROUP) steps32<N + 1>(ax, ay, az, a_ok, b, thr, a_pos, b_pos0, q, qn);
}

__global__ __launch_bounds__(MT) void k_match32(MatchArgs a, OutArgs o) {
  __shared__ uint2 s_q[WAVES][QCAP];
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t row = lane >> 4, l16 = lane & 15u;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t grp = (blk * WAVES + w) * 4u + row;
  uint2* q = s_q[w];
  uint32_t qn = 0;

  const uint32_t na = a.na.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  const bool grp_ok = grp < ngroups;
  const GroupRanges* R = grp_ok ? a.ranges + grp : nullptr;
  const uint32_t a_pos = grp * GROUP + l16;
  bool a_ok = grp_ok && a_pos < na;
  // reference cell: the group's first A source
  double c0x = 0.0, c0y = 0.0, c0z = 0.0;
  if (grp_ok) cell_centre(a, a.keysA[grp * GROUP], c0x, c0y, c0z);
  float ax = 0.f, ay = 0.f, az = 0.f;
  if (a_ok) {
    Rec32 A = a.recA32[a_pos];
    double cx, cy, cz;
    cell_centre(a, a.keysA[a_pos], cx, cy, cz);
    ax = A.x + (float)(cx - c0x);
    ay = A.y + (float)(cy - c0y);
    az = A.z + (float)(cz - c0z);
    if (a.skip_halo_a && (A.idx & HALO_BIT)) a_ok = false;
  }
  const float thr = grp_ok ? R->thr32 : 0.0f;
  Cursor c;
  c.ri = 0;
  cursor_seek(c, R);
  while (__ballot(c.active)) {
    float3 b = make_float3(1e30f, 1e30f, 1e30f);
    uint32_t b0 = c.pos;
    if (c.active && c.pos + l16 < c.end) {
      const uint32_t p = c.pos + l16;
      Rec32 B = a.recB32[p];
      double cx, cy, cz;
      cell_centre(a, a.keysB[p], cx, cy, cz);
      b = make_float3(B.x + (float)(cx - c0x), B.y + (float)(cy - c0y), B.z + (float)(cz - c0z));
    }
    steps32<0>(ax, ay, az, a_ok && c.active, b, thr, a_pos, b0, q, qn);
    if (c.active) cursor_advance(c, R);
    if (qn >= 64) {
      flush32(a, o, q, qn);
      qn = 0;
    }
  }
  if (qn) flush32(a, o, q, qn);
}

// ---------------------------------------------------------------------------
// band list: FP64 haversine from the original coordinates, double-double
// inside the FP64 band (true ties within TIE_REL of r count as matches)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_certify(const double* __restrict__ a_ra,
                                                 const double* __restrict__ a_dec,
                                                 const double* __restrict__ b_ra,
                                                 const double* __restrict__ b_dec, double r_arcsec,
                                                 double H_lo, double H_hi, Radii rad, OutArgs o) {
  unsigned long long n = o.cnt->n_band;
  if (n > o.band_cap) n = o.band_cap;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    uint2 e = o.band[i];
    double ra1 = a_ra[e.x], de1 = a_dec[e.x], ra2 = b_ra[e.y], de2 = b_dec[e.y];
    double h = haversine64(ra1, de1, ra2, de2);
    double Hlo = H_lo, Hhi = H_hi;
    if (rad.a_err) {
      const double ea = rad.a_err[e.x], eb = rad.b_err[e.y];
      pair_hav_thr(rad.k * sqrt(ea * ea + eb * eb), Hlo, Hhi);
    }
    bool in = false;
    double sep = 0.0;
    if (h < Hlo) {
      in = true;
      sep = 2.0 * asin(sqrt(h)) * RAD2ARCSEC;
    } else if (h <= Hhi) {
      dd hd = haversine_dd(ra1, de1, ra2, de2);
      dd Hd = rad.a_err ? threshold_pair_dd(rad.k, rad.a_err[e.x], rad.b_err[e.y]) : threshold_dd(r_arcsec);
      dd diff = dd_add(hd, dd_neg(Hd));
      atomicAdd(&o.cnt->n_ties, 1ull);
      if (diff.hi <= TIE_REL * Hd.hi) {
        in = true;
        sep = 2.0 * asin(sqrt(hd.hi)) * RAD2ARCSEC;
      }
    }
    if (in) emit_one(e.x, e.y, sep, o);
  }
}

__global__ void k_regions_reset(Regions reg) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NREG) {
    reg.fill[i * REG_STRIDE] = 0ull;
    reg.cand[i * REG_STRIDE] = 0ull;
  }
}

// Block k packs region k after the regions before it; block 0 also writes
// the totals. Contents beyond the caller's capacity are dropped (the call
// then reports the required count).
__global__ __launch_bounds__(256) void k_compact(OutArgs o) {
  __shared__ unsigned long long s_off;
  const uint32_t k = blockIdx.x;
  if (threadIdx.x < 64) {
    unsigned long long off = 0, tot = 0, cand = 0, mx = 0;
    for (uint32_t i = threadIdx.x; i < NREG; i += 64) {
      const unsigned long long f = o.reg.fill[i * REG_STRIDE];
      const unsigned long long used = f < o.reg.S ? f : o.reg.S;
      if (i < k) off += used;
      tot += f;
      cand += o.reg.cand[i * REG_STRIDE];
      mx = f > mx ? f : mx;
    }
    for (int d = 32; d > 0; d >>= 1) {
      off += __shfl_xor(off, d);
      tot += __shfl_xor(tot, d);
      cand += __shfl_xor(cand, d);
      const unsigned long long om = __shfl_xor(mx, d);
      mx = om > mx ? om : mx;
    }
    if (threadIdx.x == 0) {
      s_off = off;
      if (k == 0) {
        o.cnt->n_pairs = tot;
        o.cnt->n_cand = cand;
        o.cnt->region_max = mx;
      }
    }
  }
  __syncthreads();
  const unsigned long long f = o.reg.fill[k * REG_STRIDE];
  const unsigned long long n = f < o.reg.S ? f : o.reg.S;
  const unsigned long long off = s_off;
  for (unsigned long long j = threadIdx.x; j < n; j += blockDim.x) {
    const unsigned long long dst = off + j;
    if (dst >= o.cap) break;
    const unsigned long long src = (unsigned long long)k * o.reg.S + j;
    o.pairs[dst] = o.reg.pairs[src];
    if (o.sep) o.sep[dst] = o.reg.sep[src];
  }
}

}  // namespace

void launch_regions_reset(const OutArgs& o, hipStream_t s) { k_regions_reset<<<1, NREG, 0, s>>>(o.reg); }

void launch_compact(const OutArgs& o, hipStream_t s) { k_compact<<<NREG, 256, 0, s>>>(o); }

void launch_match64(const MatchArgs& a, const OutArgs& o, hipStream_t s) {
  uint32_t ngroups = (a.na.cap + GROUP - 1) / GROUP;
  if (ngroups == 0) return;
  uint32_t blocks = (ngroups + 4 * WAVES - 1) / (4 * WAVES);
  k_match64<<<blocks, MT, 0, s>>>(a, o);
}

void launch_match32(const MatchArgs& a, const OutArgs& o, hipStream_t s) {
  uint32_t ngroups = (a.na.cap + GROUP - 1) / GROUP;
  if (ngroups == 0) return;
  uint32_t blocks = (ngroups + 4 * WAVES - 1) / (4 * WAVES);
  k_match32<<<blocks, MT, 0, s>>>(a, o);
}

void launch_certify(const double* a_ra, const double* a_dec, const double* b_ra,
                    const double* b_dec, double r_arcsec, double H_lo, double H_hi,
                    const Radii& rad, const OutArgs& o, hipStream_t s) {
  k_certify<<<256, 256, 0, s>>>(a_ra, a_dec, b_ra, b_dec, r_arcsec, H_lo, H_hi, rad, o);
}

}  // namespace hlc
