// match.hip -- the distance kernels of the cross-match (the paper's kernel
// module, sections 3.1 and 4.3.1), redesigned for CDNA4 wave64.
//
// Work unit: a group of 16 consecutive A sources in (zone, RA-bin) order, one
// source per lane of a 16-lane DPP row; a wave holds four groups. A group's
// B work is the concatenation of at most MAXR ranges of the sorted B records
// (its Dec zone, RA window split at the seam, whole ring near a pole), taken
// sixteen at a time: lane l of the row loads item 16c + l of the
// concatenation, the next chunk's load is issued before the current chunk is
// tested, and DPP row_newbcast hands each of the sixteen B records to every
// lane of the row, so every A meets every B without LDS traffic.
//
// A lane collects the outcomes of its sixteen tests in a bit mask; the set
// bits (rare: about one hit per A) are drained into a small per-wave LDS
// queue, which is appended to the wave's candidate region with one atomic.
// A second kernel certifies the candidates with all lanes busy, so the
// filter loop keeps the register budget of a high-occupancy kernel. The paper
// writes a dense "1" matrix per calculation block (section 4.3.2); here only
// candidates are stored and only pairs are written.
//
// Filters (both end in the same exact decision):
//   FP64: chord^2 = |u_a - u_b|^2 of FP64 unit vectors. Candidates are pairs
//     with chord^2 <= t_hi64; below t_lo64 the pair is certainly in and its
//     separation is 2 asin(chord/2). Between the two it goes to the band list.
//   FP32: the same test in FP32 on offsets from a centre c of each group (the
//     FP32 lattice corner of its middle A entry's unit vector): every record
//     holds its unit vector as an FP32 lattice corner plus a fixed-point
//     offset inside that cell (CellRec32); a lane forms a' = (corner - c) +
//     offset for its A entry once per item, the lane that loads a B record
//     forms b' the same way once per chunk, and the tests subtract and square
//     these small offsets. The bound each lane tests against covers the
//     rounding (below); every candidate is then certified with the FP64
//     haversine of its (ra, dec), and only those within the FP64 band of r go
//     to the band list.
//
// FP64 chord error budget (u = 2^-53): each unit-vector component is a
// product of two degree-reduced sin/cos values (each within 1.5 ulp: the
// Taylor-series evaluation of sincos_small) and has an absolute error <= 4u;
// a chord component then errs by <= 8u + u|d|, so |chord_fp64 - chord| <=
// sqrt(3)*8u + u*chord ~= 1.6e-15. ETA64 = 4e-15 is used for the thresholds
// (a 2.5x margin).
//
// FP32 filter budget (v = 2^-24 the FP32 unit roundoff, w = 2^-34 the cell
// unit). A record's stored position p lies below the FP64 unit vector by
// less than w on every axis, so two entries' stored positions differ from
// their true difference by less than sqrt(3) w. Forming a' = fl(fl(corner -
// c) + count w) costs at most v(|corner - c| + |a'|) per axis, the
// difference of two offsets v|a' - b'| per axis, and the three products and
// sums of its square (1 + v)^3. For a true pair (chord <= c_r) the B entry
// lies within |a'| + c_r + sqrt(3) w of c, which bounds its own terms, so
//   |a' - b'| <= c_r + E,  E = sqrt(3) w + v (4 |a'| + 2 c_r + 7 w) + 2e-15
// (the last term: the FP64 unit vectors' own error),
// and the computed chord^2 is at most (c_r + E)^2 (1 + v)^5. Each lane tests
// against (c_r32 + E')^2 (1 + 2^-18) with c_r32 >= c_r and E' >= E evaluated
// from the norm of its own a' (with margins for the FP32 evaluation of the
// bound itself), so no true pair is rejected. With c at the middle entry of
// a group, |a'| is at most the group's half extent: at 10M x 10M sources and
// r = 2 arcsec the bound admits chords about 1e-4 r beyond r, where an FP32
// filter on unit vectors needs about 0.04 arcsec.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "hlc_kernels.hpp"

namespace hlc {

namespace {

constexpr int MT = 256;     // threads per block
constexpr int WAVES = MT / 64;
constexpr int QCAP = 256;   // per-wave candidate queue, staged above QCAP - 64
constexpr unsigned long long CAND_BLOCKS_MAX = 8192;  // grid cap of the certification walk

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
// certification of one staged candidate
// ---------------------------------------------------------------------------
struct Decision {
  bool in, band;
  uint32_t ia, ib;
  double sep;
};

template <bool HP>
__device__ inline Decision certify64(const MatchArgs& a, const Cand& c) {
  Decision v{false, false, 0u, 0u, 0.0};
  const Rec64 B = a.recB64[c.b];
  const double dx = c.u0 - B.x, dy = c.u1 - B.y, dz = c.u2 - B.z;
  const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
  v.ia = HP ? (a.recA64[c.ia].idx & IDX_MASK) : c.ia;
  v.ib = B.idx & IDX_MASK;
  bool keep = !a.self_only || v.ia < v.ib;
  if constexpr (HP) {
    // paper-scheme emulation: count the pair in the smallest shared pixel
    uint32_t pa[5], pb[5];
    const double2 ca = a.radecA[c.ia], cb = a.radecB[c.b];
    const int na_ = hp_quad(a.hp_order, ca.x, ca.y, a.hp_R, pa);
    const int nb_ = hp_quad(a.hp_order, cb.x, cb.y, a.hp_R, pb);
    uint32_t first = 0xffffffffu;
    for (int u = 0; u < na_; ++u)
      for (int w = 0; w < nb_; ++w)
        if (pa[u] == pb[w] && pa[u] < first) first = pa[u];
    keep = keep && first == a.keysA[c.ia];
  }
  double tlo = a.t_lo64, thi = a.t_hi64;
  if (a.a_err) pair_chord_thr(pair_radius(a, v.ia, v.ib), tlo, thi);
  v.in = keep && d2 <= tlo;
  v.band = keep && !v.in && d2 <= thi;
  if (v.in) v.sep = 2.0 * asin(0.5 * sqrt(d2)) * RAD2ARCSEC;
  return v;
}

__device__ inline Decision certify32(const MatchArgs& a, const Cand& c) {
  Decision v{false, false, 0u, 0u, 0.0};
  const uint32_t ia = c.ia, ib = c.b;
  // B's (ra, dec) at its sorted position when sorted, else by original index
  const double2 pb = a.radecB ? a.radecB[c.bpos] : a.srcradB[ib];
  const double2 pa = (c.u0 == c.u0) ? make_double2(c.u0, c.u1) : a.srcradA[ia];
  v.ia = ia;
  v.ib = ib;
  const double h = haversine64(pa.x, pa.y, pb.x, pb.y);
  const bool keep = !a.self_only || v.ia < v.ib;
  double Hlo = a.H_lo, Hhi = a.H_hi;
  if (a.a_err) pair_hav_thr(pair_radius(a, v.ia, v.ib), Hlo, Hhi);
  v.in = keep && h < Hlo;
  v.band = keep && !v.in && h <= Hhi;
  if (v.in) v.sep = 2.0 * asin(sqrt(h)) * RAD2ARCSEC;
  return v;
}

// Exclusive prefix of the staged candidate counts (region order), for k_cand;
// with cnt, also the candidate totals (else the compaction writes them).
__global__ __launch_bounds__(NREG) void k_cand_prefix(Regions reg, Counters* cnt) {
  __shared__ unsigned long long s[NREG];
  __shared__ unsigned long long s_max[NREG / 64];
  const uint32_t t = threadIdx.x;
  const unsigned long long f = reg.cfill[t * REG_STRIDE];
  if (cnt) {
    unsigned long long mx = f;
    for (int d = 32; d > 0; d >>= 1) {
      const unsigned long long x = __shfl_xor(mx, d);
      mx = x > mx ? x : mx;
    }
    if ((t & 63) == 0) s_max[t >> 6] = mx;
  }
  s[t] = f;
  __syncthreads();
  if (cnt && t == 0) {
    unsigned long long tot = 0, mx = 0;
    for (uint32_t i = 0; i < NREG; ++i) tot += s[i];
    for (uint32_t i = 0; i < NREG / 64; ++i) mx = s_max[i] > mx ? s_max[i] : mx;
    cnt->n_cand = tot;
    cnt->cand_max = mx;
  }
  __syncthreads();
  s[t] = f < reg.Sc ? f : reg.Sc;
  __syncthreads();
  for (uint32_t d = 1; d < NREG; d <<= 1) {
    const unsigned long long x = t >= d ? s[t - d] : 0ull;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  reg.cpre[t + 1] = s[t];
  if (t == 0) reg.cpre[0] = 0ull;
}

// Every staged candidate, regions in order: ITEMS per thread, their loads
// in flight together, then the emissions.
constexpr int CAND_ITEMS = 4;

// The pairs of one round of a block (lanes with v[j].in), written straight
// into the caller's buffer at places taken with one atomic on the pair count
// per block and round; slots past the capacity are counted, not written.
// Every thread of the block calls it (two barriers). s_wc and s_base belong
// to this round; rounds alternate between two sets, so that a wave still
// reading one round's set is never overtaken by the next round's writes.
template <int ITEMS>
__device__ inline void emit_block(const Decision (&v)[ITEMS], const OutArgs& o, uint32_t* s_wc,
                                  unsigned long long* s_base) {
  const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t m[ITEMS];
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    m[j] = __ballot(v[j].in);
    c += (uint32_t)__popcll(m[j]);
  }
  if (lane_id() == 0) s_wc[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (uint32_t i = 0; i < nw; ++i) tot += s_wc[i];
    *s_base = tot ? atomicAdd(&o.cnt->n_pairs, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  unsigned long long at = *s_base;
  for (uint32_t i = 0; i < w; ++i) at += s_wc[i];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (v[j].in) {
      const unsigned long long slot = at + rank_in(m[j]);
      if (slot < o.cap) {
        o.pairs[slot] = make_uint2(v[j].ia, v[j].ib);
        if (o.sep) o.sep[slot] = v[j].sep;
      }
    }
    at += (unsigned long long)__popcll(m[j]);
  }
}

template <bool F32, bool HP, int ITEMS>
__global__ __launch_bounds__(256) void k_cand(MatchArgs a, OutArgs o) {
  __shared__ unsigned long long s_pre[NREG + 1];
  __shared__ uint32_t s_wc[2][256 / 64];
  __shared__ unsigned long long s_base[2];
  const uint32_t t = threadIdx.x;
  for (uint32_t k = t; k <= NREG; k += blockDim.x) s_pre[k] = o.reg.cpre[k];
  __syncthreads();
  const unsigned long long total = s_pre[NREG];
  const unsigned long long tile = (unsigned long long)ITEMS * blockDim.x;
  uint32_t round = 0;
  // uniform trip count (the same for the whole block) so every lane takes
  // part in the ballots and every thread in the barriers
  for (unsigned long long base = (unsigned long long)blockIdx.x * tile; base < total;
       base += (unsigned long long)gridDim.x * tile, round ^= 1u) {
    Decision v[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const unsigned long long i = base + (unsigned long long)j * blockDim.x + t;
      v[j] = Decision{false, false, 0u, 0u, 0.0};
      if (i < total) {
        uint32_t lo = 0, hi = NREG;  // region k with s_pre[k] <= i < s_pre[k + 1]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_pre[mid] <= i) lo = mid; else hi = mid;
        }
        const unsigned long long at = (unsigned long long)lo * o.reg.Sc + (i - s_pre[lo]);
        if constexpr (F32) {
          v[j] = certify32(a, o.reg.cand[at]);
        } else {
          v[j] = certify64<HP>(a, o.reg.cand[at]);
        }
      }
    }
    if (o.direct) {
      emit_block<ITEMS>(v, o, s_wc[round], &s_base[round]);
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) emit_band(v[j].band, v[j].ia, v[j].ib, o);
    } else {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        emit_wave(v[j].in, v[j].ia, v[j].ib, v[j].sep, o);
        emit_band(v[j].band, v[j].ia, v[j].ib, o);
      }
    }
  }
}

// A wave's queue of (A position, B position) appended to its candidate
// region as self-contained records. Every queued A position belongs to the
// wave's current item, so its A data comes from the owning lane (A position
// mod 64). Entries whose B record lies in another zone (pixel) than the A
// entry are dropped here: a group straddling two zones also scans the other
// one, whose B entries include copies of sources the A entry meets in its
// own zone. One atomic per 64 entries.
// Per-lane A data of the current item, kept in LDS (not registers) until a
// candidate of that lane is staged.
struct ALane {
  double u0, u1, u2;
  uint32_t ia, key;
};

template <bool F32>
__device__ inline void stage_candidates(const MatchArgs& a, const OutArgs& o, const uint2* q, uint32_t qn,
                                        const ALane* al) {
  const uint32_t k = wave_region();
  const uint32_t lane = lane_id();
  for (uint32_t b0 = 0; b0 < qn; b0 += 64) {
    const uint32_t e = b0 + lane;
    const uint2 ent = e < qn ? q[e] : make_uint2(lane, 0u);
    const ALane& A = al[ent.x & 63u];
    const bool keep = e < qn && same_zone(a.geom, A.key, a.keysB[ent.y]);
    const uint64_t m = __ballot(keep);
    if (m == 0) continue;
    const uint32_t leader = (uint32_t)__builtin_ctzll(m);
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(&o.reg.cfill[k * REG_STRIDE], (unsigned long long)__popcll(m));
    base = __shfl(base, (int)leader);
    if (keep) {
      const unsigned long long slot = base + rank_in(m);
      const unsigned long long at = (unsigned long long)k * o.reg.Sc + slot;
      if (slot < o.reg.Sc) {
        // FP32 form: A's (ra, dec) (NaN: not at hand), B's position and the
        // two original indices (the halo bit dropped); FP64: A's unit
        // vector, A's index and B's position
        Cand c;
        c.u0 = A.u0;
        c.u1 = A.u1;
        c.ia = A.ia;
        if constexpr (F32) {
          c.u2 = 0.0;
          c.bpos = ent.y;
          c.b = a.valsB[ent.y] & IDX_MASK;
        } else {
          c.u2 = A.u2;
          c.b = ent.y;
        }
        o.reg.cand[at] = c;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// the filter
// ---------------------------------------------------------------------------
// A group's ranges as one concatenated sequence of B positions.
struct Flat {
  uint32_t s0, s1, s2, s3;  // range starts
  uint32_t p1, p2, p3;      // running lengths after ranges 0, 1, 2
  uint32_t total;
};

__device__ inline uint32_t flat_pos(const Flat& f, uint32_t t) {
  uint32_t pos = f.s0 + t;
  pos = t >= f.p1 ? f.s1 + (t - f.p1) : pos;
  pos = t >= f.p2 ? f.s2 + (t - f.p2) : pos;
  pos = t >= f.p3 ? f.s3 + (t - f.p3) : pos;
  return pos;
}

template <typename V>
struct Vec3 {
  V x, y, z;
};

// A B entry as loaded, before it is turned into the values the tests use:
// the FP64 unit vector, or the FP32 cell record.
template <bool F32>
struct RawB;
template <>
struct RawB<false> {
  double x, y, z;
};
template <>
struct RawB<true> {
  CellRec32 c;
};

template <bool F32>
__device__ inline RawB<F32> load_b(const MatchArgs& a, uint32_t p) {
  if constexpr (F32) {
    return RawB<true>{a.recB32[p]};
  } else {
    const Rec64 r = a.recB64[p];
    return RawB<false>{r.x, r.y, r.z};
  }
}

// The values the tests use: the FP64 unit vector, or the FP32 offset from
// the row's centre (cx, cy, cz); `far` for a slot past the row's sequence.
template <bool F32>
__device__ inline Vec3<typename std::conditional<F32, float, double>::type> b_values(const RawB<F32>& r, bool ok,
                                                                                     float cx, float cy, float cz) {
  using V = typename std::conditional<F32, float, double>::type;
  const V far = (V)1e30;
  Vec3<V> B{far, far, far};
  if constexpr (F32) {
    float ox, oy, oz;
    cell_offset(r.c, cx, cy, cz, ox, oy, oz);
    if (ok) B = Vec3<V>{ox, oy, oz};
  } else {
    (void)cx;
    (void)cy;
    (void)cz;
    if (ok) B = Vec3<V>{r.x, r.y, r.z};
  }
  return B;
}

// up to sixteen tests: bit N of mask <- |a - b_N|^2 <= thr, b_N the record of
// lane N of this lane's row; steps from nmax (wave-uniform: no row has a
// record there) on are skipped
template <int N, typename V>
__device__ inline void tests(const Vec3<V>& A, const Vec3<V>& B, V thr, uint32_t nmax, uint32_t& mask) {
  if (N >= nmax) return;
  const V dx = A.x - row_bcast<N>(B.x);
  const V dy = A.y - row_bcast<N>(B.y);
  const V dz = A.z - row_bcast<N>(B.z);
  const V d2 = fma(dx, dx, fma(dy, dy, dz * dz));
  mask |= (d2 <= thr ? 1u : 0u) << N;
  if constexpr (N + 1 < GROUP) tests<N + 1, V>(A, B, thr, nmax, mask);
}

// Loads of one work item (four groups, one per row) that do not depend on
// other loads: the group's ranges and the A entry's source index.
struct ItemHead {
  uint32_t s[MAXR], e[MAXR], n;
  uint32_t grp, a_pos, va;
  bool a_ok;
};

__device__ inline ItemHead item_head(const MatchArgs& a, uint32_t item, uint32_t row, uint32_t l16, uint32_t na,
                                     uint32_t ngroups) {
  ItemHead h;
  h.grp = item * 4u + row;
  h.a_pos = h.grp * GROUP + l16;
  const bool grp_ok = h.grp < ngroups;
  h.a_ok = grp_ok && h.a_pos < na;
  h.n = 0u;
#pragma unroll
  for (int t = 0; t < MAXR; ++t) h.s[t] = h.e[t] = 0u;
  if (grp_ok) {
    const GroupRanges* R = a.ranges + h.grp;
    h.n = R->count;
#pragma unroll
    for (int t = 0; t < MAXR; ++t) {
      h.s[t] = R->start[t];
      h.e[t] = R->end[t];
    }
  }
  h.va = (h.a_ok && a.valsA) ? a.valsA[h.a_pos] : 0u;
  return h;
}

__device__ inline Flat flatten(const ItemHead& h) {
  auto len = [&](int t) { return (uint32_t)t < h.n && h.e[t] > h.s[t] ? h.e[t] - h.s[t] : 0u; };
  Flat f;
  f.s0 = h.s[0];
  f.s1 = h.s[1];
  f.s2 = h.s[2];
  f.s3 = h.s[3];
  f.p1 = len(0);
  f.p2 = f.p1 + len(1);
  f.p3 = f.p2 + len(2);
  f.total = f.p3 + len(3);
  return f;
}

// What a lane reads of its A entry: the FP32 cell record or the FP64 unit
// vector, what its staged candidates carry (u0..u2) and its key.
struct ARaw {
  CellRec32 ca;
  double u0, u1, u2;
  uint32_t key;
};

template <bool F32>
__device__ inline ARaw load_a(const MatchArgs& a, const ItemHead& h) {
  ARaw r{{0.f, 0.f, 0.f, 0u}, 0.0, 0.0, 0.0, 0u};
  if (!h.a_ok) return r;
  r.key = a.keysA[h.a_pos];
  const uint32_t idx = h.va;  // the entry's source index (halo bit included)
  if constexpr (F32) {
    if (a.a_in_place) {
      // (ra, dec) in place; the cell record as the layout would write it
      const double2 p = a.srcradA[idx & IDX_MASK];
      double x, y, z;
      unit_vector(p.x, p.y, x, y, z);
      r.ca = encode_cell(x, y, z);
      r.u0 = p.x;
      r.u1 = p.y;
    } else {
      r.ca = a.recA32[h.a_pos];
      if (a.radecA) {
        const double2 p = a.radecA[h.a_pos];
        r.u0 = p.x;
        r.u1 = p.y;
      } else {
        r.u0 = __builtin_nan("");  // the certification reads A's (ra, dec)
      }
    }
  } else {
    if (a.a_in_place) {
      // (ra, dec) in place; the unit vector as the layout would write it
      const double2 p = a.srcradA[idx & IDX_MASK];
      unit_vector(p.x, p.y, r.u0, r.u1, r.u2);
    } else {
      const Rec64 s = a.recA64[h.a_pos];
      r.u0 = s.x;
      r.u1 = s.y;
      r.u2 = s.z;
    }
  }
  return r;
}

// Persistent: wave w of W takes items w, w + W, ... (an item is four groups,
// one per 16-lane row). The next item's ranges and A index are loaded
// while the current one is tested, and its A records once the current one's
// chunks are done (their loads then overlap the drain of the queue).
template <bool F32>
__global__ __launch_bounds__(MT, 7) void k_filter(MatchArgs a, OutArgs o) {
  using V = typename std::conditional<F32, float, double>::type;
  __shared__ uint2 s_q[WAVES][QCAP];
  __shared__ ALane s_a[WAVES][64];
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t row = lane >> 4, l16 = lane & 15u;
  // consecutive logical blocks on one XCD: neighbouring groups share B
  // records in its L2
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t W = gridDim.x * WAVES;
  uint2* q = s_q[w];
  uint32_t qn = 0;

  const uint32_t na = a.na.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  const uint32_t nitems = (ngroups + 3u) / 4u;
  const V far = (V)1e30;

  uint32_t item = blk * WAVES + w;
  ItemHead head = item_head(a, item, row, l16, na, ngroups);
  ARaw ar = load_a<F32>(a, head);
  while (__builtin_amdgcn_readfirstlane(item) < nitems) {
    const ItemHead cur = head;
    const uint32_t next = item + W;
    // stage 1 of this item: its first B chunk (its A record is in flight)
    const Flat f = flatten(cur);
    uint32_t t = l16;
    uint32_t bp = t < f.total ? flat_pos(f, t) : 0u;
    RawB<F32> rb{};
    if (t < f.total) rb = load_b<F32>(a, bp);
    bool a_ok = cur.a_ok;
    // what a staged candidate carries of this lane's A entry
    const uint32_t ia = !a_ok ? 0u : (a.hp_order >= 0 ? cur.a_pos : (cur.va & IDX_MASK));
    if (a_ok && a.skip_halo_a && (cur.va & HALO_BIT)) a_ok = false;
    s_a[w][lane] = ALane{ar.u0, ar.u1, ar.u2, ia, ar.key};
    const CellRec32 ca = ar.ca;
    const Vec3<double> a64{ar.u0, ar.u1, ar.u2};
    // FP32: the row's centre is the lattice corner of its middle entry (its
    // first when the group has eight entries or fewer); each lane's offset
    // from it and the bound covering the filter's rounding (header comment)
    float cx = 0.f, cy = 0.f, cz = 0.f;
    Vec3<V> A{-far, -far, -far};
    V thr;
    if constexpr (F32) {
      const bool mid = cur.grp * GROUP + 8u < na;
      const float mx = row_bcast<8>(ca.x), my = row_bcast<8>(ca.y), mz = row_bcast<8>(ca.z);
      const float fx = row_bcast<0>(ca.x), fy = row_bcast<0>(ca.y), fz = row_bcast<0>(ca.z);
      cx = mid ? mx : fx;
      cy = mid ? my : fy;
      cz = mid ? mz : fz;
      float ax, ay, az;
      cell_offset(ca, cx, cy, cz, ax, ay, az);
      // E' >= sqrt(3) w + v (4 |a'| + 2 c_r + 7 w) + 2e-15 (the FP64 unit
      // vectors' own error): the factors 4.01 and 2.01 and the added 2^-30 v
      // cover the FP32 evaluation of |a'| and of this bound
      const float an = sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az)));
      const float E = 0x1.bb68p-34f + 2e-15f + 0x1p-24f * (4.01f * an + 2.01f * a.c_r32 + 0x1p-30f);
      const float cr = a.c_r32 + E;
      thr = cr * cr * (1.0f + 0x1p-18f);
      if (a_ok) A = Vec3<V>{ax, ay, az};
    } else {
      thr = a.t_hi64;
      if (a_ok) A = Vec3<V>{a64.x, a64.y, a64.z};
    }
    // stage 0 of the next item, in flight while this one is tested
    head = item_head(a, next, row, l16, na, ngroups);

    // chunk c of the row covers items [16c, 16c + 16) of the concatenation;
    // the wave runs as many chunks as its longest row needs (scalar)
    const uint32_t tmax = max(max((uint32_t)__builtin_amdgcn_readlane((int)f.total, 0),
                                  (uint32_t)__builtin_amdgcn_readlane((int)f.total, 16)),
                              max((uint32_t)__builtin_amdgcn_readlane((int)f.total, 32),
                                  (uint32_t)__builtin_amdgcn_readlane((int)f.total, 48)));
    const uint32_t nch = (tmax + 15u) >> 4;
    for (uint32_t c = 0; c < nch; ++c) {
      // next chunk's record in flight while this one is tested
      const uint32_t tn = t + GROUP;
      const uint32_t bpn = tn < f.total ? flat_pos(f, tn) : 0u;
      RawB<F32> rbn{};
      if (tn < f.total) rbn = load_b<F32>(a, bpn);
      const Vec3<V> B = b_values<F32>(rb, t < f.total, cx, cy, cz);

      // records in this chunk: the largest count over the wave's four rows
      const uint32_t nmax = min(tmax - 16u * c, (uint32_t)GROUP);
      uint32_t mask = 0u;
      tests<0, V>(A, B, thr, nmax, mask);
      // drain the hits into the queue, lowest bit first
      while (__ballot(mask != 0u)) {
        const bool has = mask != 0u;
        const uint32_t bit = has ? (uint32_t)__builtin_ctz(mask) : 0u;
        const uint32_t bpos = (uint32_t)__shfl((int)bp, (int)((lane & 48u) | bit));
        const uint64_t m = __ballot(has);
        if (has) q[qn + rank_in(m)] = make_uint2(cur.a_pos, bpos);
        qn += (uint32_t)__popcll(m);
        mask &= mask - 1u;
        if (qn > QCAP - 64) {
          stage_candidates<F32>(a, o, q, qn, s_a[w]);
          qn = 0;
        }
      }
      t = tn;
      bp = bpn;
      rb = rbn;
    }
    ar = load_a<F32>(a, head);
    // the queue holds this item's entries only (their A data is in its lanes)
    if (qn) {
      stage_candidates<F32>(a, o, q, qn, s_a[w]);
      qn = 0;
    }
    item = next;
  }
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
    reg.cfill[i * REG_STRIDE] = 0ull;
  }
}

// Blocks k * CPB .. k * CPB + CPB - 1 pack region k after the regions
// before it; block 0 also writes the totals. Contents beyond the caller's
// capacity are dropped (the call then reports the required count).
constexpr uint32_t CPB = 16;  // blocks per region

__global__ __launch_bounds__(256) void k_compact(OutArgs o) {
  __shared__ unsigned long long s_off;
  const uint32_t k = blockIdx.x / CPB, part = blockIdx.x % CPB;
  if (threadIdx.x < 64) {
    unsigned long long off = 0, tot = 0, cand = 0, mx = 0, cmx = 0;
    for (uint32_t i = threadIdx.x; i < NREG; i += 64) {
      const unsigned long long f = o.reg.fill[i * REG_STRIDE];
      const unsigned long long c = o.reg.cfill[i * REG_STRIDE];
      const unsigned long long used = f < o.reg.S ? f : o.reg.S;
      if (i < k) off += used;
      tot += f;
      cand += c;
      mx = f > mx ? f : mx;
      cmx = c > cmx ? c : cmx;
    }
    for (int d = 32; d > 0; d >>= 1) {
      off += __shfl_xor(off, d);
      tot += __shfl_xor(tot, d);
      cand += __shfl_xor(cand, d);
      const unsigned long long om = __shfl_xor(mx, d), oc = __shfl_xor(cmx, d);
      mx = om > mx ? om : mx;
      cmx = oc > cmx ? oc : cmx;
    }
    if (threadIdx.x == 0) {
      s_off = off;
      if (blockIdx.x == 0) {
        o.cnt->n_pairs = tot;
        o.cnt->n_cand = cand;
        o.cnt->region_max = mx;
        o.cnt->cand_max = cmx;
      }
    }
  }
  __syncthreads();
  const unsigned long long f = o.reg.fill[k * REG_STRIDE];
  const unsigned long long n = f < o.reg.S ? f : o.reg.S;
  const unsigned long long off = s_off;
  for (unsigned long long j = (unsigned long long)part * blockDim.x + threadIdx.x; j < n;
       j += (unsigned long long)CPB * blockDim.x) {
    const unsigned long long dst = off + j;
    if (dst >= o.cap) break;
    const unsigned long long src = (unsigned long long)k * o.reg.S + j;
    o.pairs[dst] = o.reg.pairs[src];
    if (o.sep) o.sep[dst] = o.reg.sep[src];
  }
}

}  // namespace

void launch_regions_reset(const OutArgs& o, hipStream_t s) { k_regions_reset<<<1, NREG, 0, s>>>(o.reg); }

void launch_compact(const OutArgs& o, hipStream_t s) { k_compact<<<NREG * CPB, 256, 0, s>>>(o); }

void launch_filter(const MatchArgs& a, const OutArgs& o, bool fp32, int items_per_wave, hipStream_t s) {
  const uint32_t ngroups = (a.na.cap + GROUP - 1) / GROUP;
  if (ngroups == 0) return;
  const uint32_t items = (ngroups + 3) / 4;
  const uint32_t per_block = WAVES * (uint32_t)std::max(items_per_wave, 1);
  const uint32_t blocks = (items + per_block - 1) / per_block;
  if (fp32) k_filter<true><<<blocks, MT, 0, s>>>(a, o);
  else k_filter<false><<<blocks, MT, 0, s>>>(a, o);
}

void launch_cand(const MatchArgs& a, const OutArgs& o, bool fp32, hipStream_t s) {
  // one candidate per thread when the staging is full; the walk is
  // grid-stride beyond that
  const unsigned long long slots = (unsigned long long)NREG * o.reg.Sc;
  const uint32_t blocks = (uint32_t)std::min<unsigned long long>(
      CAND_BLOCKS_MAX, std::max(1ull, (slots + 256 * CAND_ITEMS - 1) / (256 * CAND_ITEMS)));
  k_cand_prefix<<<1, NREG, 0, s>>>(o.reg, o.direct ? o.cnt : nullptr);
  if (fp32) k_cand<true, false, CAND_ITEMS><<<blocks, 256, 0, s>>>(a, o);
  else if (a.hp_order >= 0) k_cand<false, true, 1><<<blocks, 256, 0, s>>>(a, o);
  else k_cand<false, false, CAND_ITEMS><<<blocks, 256, 0, s>>>(a, o);
}

void launch_certify(const double* a_ra, const double* a_dec, const double* b_ra,
                    const double* b_dec, double r_arcsec, double H_lo, double H_hi,
                    const Radii& rad, const OutArgs& o, hipStream_t s) {
  k_certify<<<256, 256, 0, s>>>(a_ra, a_dec, b_ra, b_dec, r_arcsec, H_lo, H_hi, rad, o);
}

}  // namespace hlc
