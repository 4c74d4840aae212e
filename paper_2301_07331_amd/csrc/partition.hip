// partition.hip -- the first level of the cross-match: both catalogues are
// grouped by declination zone and then by RA bin, on the GPU.
//
// The paper partitions on the CPU with HEALPix pixels and copies records that
// lie near a pixel edge into the neighbouring pixel (section 3.2, Algorithm 1:
// RA and Dec shifted by the error radius, so corners, the RA seam and the
// 1/cos(Dec) stretch of RA near the poles can be missed). Here:
//   * keys: zone z = floor((Dec + 90) / h), RA bin b = floor(RA * nbins / 360),
//     key = (z << rb) | b (32 bits);
//   * every B source is also keyed into the neighbouring zone when it lies
//     within r of that zone (a Dec halo), so an A source needs B from its own
//     zone only;
//   * RA neighbourhoods are bin windows of half-width asin(sin r / cos Dec*)
//     split at the 0/360 seam, and the whole zone ring within r of a pole;
//   * keys are sorted with a stable LSD radix sort written here (8-bit digits,
//     per-tile histograms, a device-wide scan, LDS-staged stable scatter).
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "hlc_kernels.hpp"

namespace hlc {

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 32;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // 8192 keys per tile
constexpr int RS_BINS = 256;
// the scatter: 512 threads, 16 keys each, per 8,192-key tile (eight waves,
// each ranking a contiguous eighth of the tile)
constexpr int SC_THREADS = 512;
constexpr int SC_ITEMS = 16;
constexpr int SC_WAVES = SC_THREADS / 64;
static_assert(SC_THREADS * SC_ITEMS == RS_TILE, "a scatter block ranks one radix tile");

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// keys and values [0, count) from one buffer pair to another
__global__ void k_copy_pairs(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                             uint32_t* __restrict__ kd, uint32_t* __restrict__ vd, DevCount nc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc.get()) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}

__global__ void k_zero_counters(Counters* c) {
  uint32_t* p = reinterpret_cast<uint32_t*>(c);
  for (uint32_t i = threadIdx.x; i < sizeof(Counters) / 4; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// keygen
// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one value per thread (NW waves of 64).
template <int NW = 4>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total, uint32_t* s_w) {
  const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    uint32_t s = s_w[k];
    if ((uint32_t)k < w) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

// Each block keys KG_ITEMS * KG_THREADS sources, one radix tile (so that it
// alone counts the tile's first-pass digits); the Dec-halo copies of the
// block are placed with a single atomic on the halo counter (one per block
// keeps the contended counter off the critical path).
constexpr int KG_ITEMS = 16;
constexpr uint32_t KG_THREADS = 512;
constexpr uint32_t KG_TILE = KG_ITEMS * KG_THREADS;
static_assert(KG_TILE == (uint32_t)RS_TILE, "a keygen block fills one radix tile");

// Besides the keys, each source's (ra, dec) is written in input order as one
// 16-B record (coalesced), when radec is given: the side's only per-source
// record. A gathered side's layout then reads one random line per entry
// (half the line traffic of two 8-B reads from the caller's arrays) and
// computes the sorted working record from it; a side that the filter reads
// in place is read once per entry there, the filter computing the record.
__global__ __launch_bounds__(KG_THREADS) void k_keygen(const double* __restrict__ ra,
                                                const double* __restrict__ dec, uint32_t n,
                                                Geom g, int halo, uint32_t err_bit,
                                                uint32_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals, Counters* cnt,
                                                double2* __restrict__ radec, uint32_t* __restrict__ hist,
                                                uint32_t hist_tiles, int hist_shift, uint32_t hist_full,
                                                int iota_vals) {
  constexpr int NW = KG_THREADS / 64;
  __shared__ uint32_t s_w[NW];
  __shared__ unsigned long long s_base;
  __shared__ uint32_t s_h[RS_BINS];
  const uint32_t t = threadIdx.x;
  // the first radix pass's digit counts of this block's keys (its radix
  // tile), stored whole when the tile holds keygen entries only (tiles below
  // hist_full; the others, which may mix in halo copies, are counted by the
  // pass's own histogram kernel)
  const uint32_t rtile = blockIdx.x;
  const bool count = hist && rtile < hist_full;
  if (count && t < (uint32_t)RS_BINS) s_h[t] = 0u;
  __syncthreads();
  const uint32_t base = blockIdx.x * KG_TILE;
  uint32_t hkey[KG_ITEMS];
  uint32_t need = 0;  // bit j: item j has a halo copy
  bool bad = false;
  // every load of the tile in flight before the first use
  double av[KG_ITEMS], dv[KG_ITEMS];
  if (base + KG_TILE <= n) {
#pragma unroll
    for (int j = 0; j < KG_ITEMS; ++j) {
      av[j] = ra[base + (uint32_t)j * KG_THREADS + t];
      dv[j] = dec[base + (uint32_t)j * KG_THREADS + t];
    }
  } else {
#pragma unroll
    for (int j = 0; j < KG_ITEMS; ++j) {
      const uint32_t i = base + (uint32_t)j * KG_THREADS + t;
      av[j] = i < n ? ra[i] : 0.0;
      dv[j] = i < n ? dec[i] : 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < KG_ITEMS; ++j) {
    const uint32_t i = base + (uint32_t)j * KG_THREADS + t;
    hkey[j] = 0u;
    if (i < n) {
      double a = av[j], d = dv[j];
      const bool ok = valid_pos(a, d);
      if (!ok) {
        bad = true;
        a = 0.0;
        d = 0.0;
      }
      const int32_t z = zone_of(g, d);
      const uint32_t b = bin_of(g, a);
      const uint32_t fr = frac_of(g, a, b);
      const uint32_t key = make_key(g, z, b) | fr;
      keys[i] = key;
      if (!iota_vals) vals[i] = i;  // (else the sort's first pass takes the position)
      if (count) atomicAdd(&s_h[(key >> hist_shift) & 0xffu], 1u);
      if (radec) radec[i] = make_double2(a, d);
      if (halo && ok) {
        // the zone height is >= 2 r, so the padded Dec window reaches at
        // most one neighbouring zone
        const int32_t zl = zone_of(g, d - g.rpad_deg), zh = zone_of(g, d + g.rpad_deg);
        const int32_t other = (zl != z) ? zl : zh;
        if (other != z) {
          hkey[j] = make_key(g, other, b) | fr;
          need |= 1u << j;
        }
      }
    }
  }
  if (bad) atomicOr(&cnt->err, err_bit);
  if (count) {
    __syncthreads();
    if (t < (uint32_t)RS_BINS) hist[(size_t)t * hist_tiles + rtile] = s_h[t];
  }
  if (!halo) return;
  uint32_t total;
  const uint32_t off = block_exclusive_scan<NW>((uint32_t)__popc(need), &total, s_w);
  if (total == 0) return;
  if (t == 0) s_base = atomicAdd(&cnt->n_halo, (unsigned long long)total);
  __syncthreads();
  uint64_t pos = (uint64_t)n + s_base + off;
#pragma unroll
  for (int j = 0; j < KG_ITEMS; ++j) {
    if (need & (1u << j)) {
      keys[pos] = hkey[j];
      vals[pos] = (base + (uint32_t)j * KG_THREADS + t) | HALO_BIT;
      ++pos;
    }
  }
}

// ---------------------------------------------------------------------------
// LSD radix sort (8-bit digits)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                           DevCount nc, int shift,
                                                           uint32_t* __restrict__ counts,
                                                           uint32_t ntiles, uint32_t tile0) {
  __shared__ uint32_t h[4][RS_BINS];
  const uint32_t n = nc.get();
  const uint32_t t = threadIdx.x, w = t >> 6;
  const uint32_t tile = tile0 + blockIdx.x;
  for (uint32_t k = t; k < 4 * RS_BINS; k += RS_THREADS) (&h[0][0])[k] = 0u;
  __syncthreads();
  const uint32_t base = tile * RS_TILE;
  // every load in flight before the first use
  uint32_t k[RS_ITEMS];
  if (base + RS_TILE <= n) {
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) k[j] = keys[base + j * RS_THREADS + t];
  } else {
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
      const uint32_t e = base + j * RS_THREADS + t;
      k[j] = e < n ? keys[e] : 0u;
    }
  }
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j)
    if (base + j * RS_THREADS + t < n) atomicAdd(&h[w][(k[j] >> shift) & 0xffu], 1u);
  __syncthreads();
  counts[t * ntiles + tile] = h[0][t] + h[1][t] + h[2][t] + h[3][t];
}

// Block d: exclusive scan, in place, of digit d's per-tile counts (tile
// order); the digit's total goes to totals[d]. The scatter adds the
// exclusive prefix of the totals, so one launch replaces a device-wide scan.
__global__ __launch_bounds__(RS_THREADS) void k_scan_digits(uint32_t* __restrict__ counts, uint32_t ntiles,
                                                            uint32_t* __restrict__ totals) {
  __shared__ uint32_t s_w[4];
  uint32_t* c = counts + (size_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (uint32_t off = 0; off < ntiles; off += RS_THREADS) {
    const uint32_t i = off + threadIdx.x;
    const uint32_t x = i < ntiles ? c[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(x, &tot, s_w);
    if (i < ntiles) c[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// One stable scatter pass over 8,192-key tiles, persistent: block b takes
// tiles b, b + G, ... of the entries present (G blocks), and the next tile's
// keys and values are loaded while the current one is ranked and written, so
// that a block's loads do not wait behind its own ranking. A tile is ranked
// in LDS (per-wave digit counts, 8 ballots per item for the lanes sharing a
// digit) and leaves in runs of consecutive positions.
__global__ __launch_bounds__(SC_THREADS) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, DevCount nc, int shift,
    const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ totals, uint32_t ntiles, uint32_t iota) {
  __shared__ uint32_t s_k[RS_TILE];
  __shared__ uint32_t s_v[RS_TILE];
  __shared__ uint32_t s_wh[SC_WAVES][RS_BINS];
  __shared__ uint32_t s_start[RS_BINS];
  __shared__ uint32_t s_goff[RS_BINS];
  __shared__ uint32_t s_dbase[RS_BINS];
  __shared__ uint32_t s_w[SC_WAVES];
  const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t n = nc.get();
  const uint32_t nt = (uint32_t)(((uint64_t)n + RS_TILE - 1) / RS_TILE);
  uint32_t tile = blockIdx.x;
  if (tile >= nt) return;  // (block-uniform)
  {
    // digit d's first position before any tile's share: the same for every tile
    uint32_t all;
    const uint32_t st = block_exclusive_scan<SC_WAVES>(t < RS_BINS ? totals[t] : 0u, &all, s_w);
    if (t < RS_BINS) s_dbase[t] = st;
  }
  auto load = [&](uint32_t tl, uint32_t (&k)[SC_ITEMS], uint32_t (&v)[SC_ITEMS], uint32_t& off) {
    const uint32_t e0 = tl * RS_TILE + w * (RS_TILE / SC_WAVES) + lane;
    off = t < RS_BINS ? offsets[t * ntiles + tl] : 0u;
    // (entries below iota carry their own position as value: not loaded)
    if (tl * RS_TILE + RS_TILE <= min(n, iota)) {
#pragma unroll
      for (int j = 0; j < SC_ITEMS; ++j) {
        k[j] = keys_in[e0 + j * 64];
        v[j] = e0 + j * 64;
      }
    } else if (tl * RS_TILE + RS_TILE <= n) {
#pragma unroll
      for (int j = 0; j < SC_ITEMS; ++j) {
        const uint32_t e = e0 + j * 64;
        k[j] = keys_in[e];
        v[j] = e < iota ? e : vals_in[e];
      }
    } else {
#pragma unroll
      for (int j = 0; j < SC_ITEMS; ++j) {
        const uint32_t e = e0 + j * 64;
        k[j] = e < n ? keys_in[e] : 0u;
        v[j] = e < n ? (e < iota ? e : vals_in[e]) : 0u;
      }
    }
  };
  uint32_t key[SC_ITEMS], val[SC_ITEMS], off;
  load(tile, key, val, off);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  while (true) {
    const uint32_t base = tile * RS_TILE;
    const uint32_t tile_n = min((uint32_t)RS_TILE, n - base);
    const uint32_t next = tile + gridDim.x;
    for (uint32_t k = t; k < SC_WAVES * RS_BINS; k += SC_THREADS) (&s_wh[0][0])[k] = 0u;
    if (t < RS_BINS) s_goff[t] = s_dbase[t] + off;
    __syncthreads();
    const uint32_t e0 = base + w * (RS_TILE / SC_WAVES) + lane;
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j)
      if (e0 + j * 64 < n) atomicAdd(&s_wh[w][(key[j] >> shift) & 0xffu], 1u);
    __syncthreads();
    {
      // digit d's start in the tile, then each wave's start within it
      const uint32_t d = t;
      uint32_t c[SC_WAVES] = {}, sum = 0u;
      if (d < RS_BINS) {
#pragma unroll
        for (int k = 0; k < SC_WAVES; ++k) {
          c[k] = s_wh[k][d];
          sum += c[k];
        }
      }
      uint32_t tot;
      const uint32_t st = block_exclusive_scan<SC_WAVES>(sum, &tot, s_w);
      if (d < RS_BINS) {
        s_start[d] = st;
        uint32_t run = st;
#pragma unroll
        for (int k = 0; k < SC_WAVES; ++k) {
          s_wh[k][d] = run;
          run += c[k];
        }
      }
    }
    __syncthreads();
    // the next tile in flight from here on
    uint32_t nkey[SC_ITEMS], nval[SC_ITEMS], noff = 0u;
    if (next < nt) load(next, nkey, nval, noff);
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) {
      const uint32_t e = e0 + j * 64;
      const bool valid = e < n;
      const uint32_t d = (key[j] >> shift) & 0xffu;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const uint64_t b = __ballot((d >> bit) & 1u);
        peers &= ((d >> bit) & 1u) ? b : ~b;
      }
      if (valid) {
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t pos = s_wh[w][d] + rank;
        s_k[pos] = key[j];
        s_v[pos] = val[j];
        if ((peers >> lane) == 1ull) s_wh[w][d] += rank + 1u;
      }
    }
    __syncthreads();
    for (uint32_t i = t; i < tile_n; i += SC_THREADS) {
      const uint32_t k = s_k[i];
      const uint32_t d = (k >> shift) & 0xffu;
      const uint32_t gpos = s_goff[d] + (i - s_start[d]);
      keys_out[gpos] = k;
      vals_out[gpos] = s_v[i];
    }
    if (next >= nt) break;
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) {
      key[j] = nkey[j];
      val[j] = nval[j];
    }
    off = noff;
    tile = next;
    __syncthreads();  // the tile's LDS is read out before the next one fills it
  }
}

// ---------------------------------------------------------------------------
// zone / cell tables
// ---------------------------------------------------------------------------
// Per zone: the RA half-width (deg, padded outward) of a window of radius
// r around any of its sources, and that width in bins plus one (-1 for
// both: the zone is scanned as a whole ring)
__device__ inline void zone_table_entry(const Geom& g, int32_t z, int32_t* __restrict__ zmarg,
                                        double* __restrict__ zdelta) {
  double lo = zone_lo(g, z);
  double hi = lo + zone_height(g, z);
  // largest |Dec| a source assigned to this zone can have (padded for the
  // rounding of the zone formula)
  double dstar = fmin(fmax(fabs(lo), fabs(hi)) + 1e-9, 90.0);
  int32_t m = -1;  // -1: whole zone ring
  double dz = -1.0;
  if (dstar + g.rpad_deg < 90.0) {
    double ss, cs, sd, cd;
    sincos_deg(g.rpad_deg, &ss, &cs);
    sincos_deg(dstar, &sd, &cd);
    double x = ss / cd;
    if (x < 0.99) {
      double delta = asin(x) * (180.0 / M_PI) * (1.0 + 1e-9) + 1e-12;
      // floor(ra * scale) is monotone in ra, and a shift by delta moves it
      // by at most ceil(delta * scale) + 1 bins (one for the rounding of
      // the product)
      double mm = ceil(delta * g.bin_scale) + 1.0;
      if (2.0 * mm + 1.0 < (double)g.nbins) {
        m = (int32_t)mm;
        dz = delta;
      }
    }
  }
  zmarg[z] = m;
  zdelta[z] = dz;
}

__global__ void k_zone_tables(Geom g, int32_t* __restrict__ zmarg, double* __restrict__ zdelta) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (uint32_t)g.nz) zone_table_entry(g, (int32_t)i, zmarg, zdelta);
}

__device__ inline uint32_t lower_bound_u32(const uint32_t* keys, uint32_t lo, uint32_t hi, uint32_t K) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] < K) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// zstart[z] = first position of zone z in the sorted keys; zstart[nz] = n
__global__ void k_zone_starts(const uint32_t* __restrict__ keys, DevCount nc, Geom g,
                              uint32_t* __restrict__ zstart) {
  const uint32_t n = nc.get();
  uint32_t z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z > (uint32_t)g.nz) return;
  if (z == (uint32_t)g.nz) { zstart[z] = n; return; }
  zstart[z] = lower_bound_u32(keys, 0, n, make_key(g, z, 0u));
}

// The same from the coarse key index when a zone's first key is a multiple
// of the index's step (idx[i] = first position with key >= i << shift).
// With zmarg, the zone tables as well (one launch for both).
__global__ void k_zone_starts_index(const uint32_t* __restrict__ idx, int shift, uint32_t T, DevCount nc, Geom g,
                                    uint32_t* __restrict__ zstart, int32_t* __restrict__ zmarg,
                                    double* __restrict__ zdelta) {
  const uint32_t n = nc.get();
  uint32_t z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z > (uint32_t)g.nz) return;
  if (z == (uint32_t)g.nz) { zstart[z] = n; return; }
  if (zmarg) zone_table_entry(g, (int32_t)z, zmarg, zdelta);
  const uint32_t i = make_key(g, (int32_t)z, 0u) >> shift;
  zstart[z] = i < T ? idx[i] : n;
}

// ---------------------------------------------------------------------------
// working layouts
// ---------------------------------------------------------------------------
// FP64 record (unit vector + the entry's value) of each sorted entry, from
// the caller's coordinates or from the keygen's interleaved (ra, dec) (il)
__global__ __launch_bounds__(256) void k_layout64(const uint32_t* __restrict__ vals, DevCount nc,
                                                  const double* __restrict__ ra,
                                                  const double* __restrict__ dec,
                                                  const double2* __restrict__ il,
                                                  Rec64* __restrict__ rec) {
  // XCD-aware over the blocks the device-side count fills (the grid covers the
  // capacity): the sources a run of sorted entries reads land in one L2
  const uint32_t n = nc.get(), nb = (n + blockDim.x - 1) / blockDim.x;
  if (blockIdx.x >= nb) return;
  const uint32_t p = xcd_block(blockIdx.x, nb) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t v = vals[p];
  uint32_t i = v & IDX_MASK;
  double a, d;
  if (il) {
    const double2 q = il[i];
    a = q.x;
    d = q.y;
  } else {
    a = ra[i];
    d = dec[i];
  }
  double x, y, z;
  unit_vector(a, d, x, y, z);
  Rec64 r;
  r.x = x;
  r.y = y;
  r.z = z;
  r.idx = v;
  r.pad = 0u;
  rec[p] = r;
}

// FP32 cell record of the FP64 unit vector (and, with radec, the (ra, dec)),
// sorted, from the caller's coordinates or from the keygen's interleaved
// (ra, dec) records (il)
__global__ __launch_bounds__(256) void k_layout32(const uint32_t* __restrict__ vals, DevCount nc,
                                                  const double* __restrict__ ra,
                                                  const double* __restrict__ dec,
                                                  const double2* __restrict__ il,
                                                  CellRec32* __restrict__ rec, double2* __restrict__ radec) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nc.get()) return;
  uint32_t i = vals[p] & IDX_MASK;
  double a, d;
  if (il) {
    const double2 q = il[i];
    a = q.x;
    d = q.y;
  } else {
    a = ra[i];
    d = dec[i];
  }
  double x, y, z;
  unit_vector(a, d, x, y, z);
  rec[p] = encode_cell(x, y, z);
  if (radec) radec[p] = make_double2(a, d);
}

// ---------------------------------------------------------------------------
// merge path: lb[i] = number of B keys strictly below keysA[i]
// ---------------------------------------------------------------------------
constexpr int MP_THREADS = 256;
constexpr int MP_ITEMS = 8;
constexpr int MP_TILE = MP_THREADS * MP_ITEMS;

// number of A elements among the first d merged elements (A first on ties)
__device__ inline uint32_t merge_split(const uint32_t* A, uint32_t na, const uint32_t* B, uint32_t nb,
                                       uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0u;
  uint32_t hi = d < na ? d : na;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (A[mid] <= B[d - mid - 1]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// The split of every tile boundary, all searches in parallel (one thread
// each), so that no merge tile waits on a search through the whole arrays.
__global__ __launch_bounds__(256) void k_merge_splits(const uint32_t* __restrict__ A, DevCount nac,
                                                      const uint32_t* __restrict__ B, DevCount nbc,
                                                      uint32_t nsplit, uint32_t* __restrict__ splits) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsplit) return;
  const uint32_t na = nac.get(), nb = nbc.get();
  const uint64_t d = min((uint64_t)t * MP_TILE, (uint64_t)na + nb);
  splits[t] = merge_split(A, na, B, nb, (uint32_t)d);
}

__global__ __launch_bounds__(MP_THREADS) void k_merge_lb(const uint32_t* __restrict__ A, DevCount nac,
                                                         const uint32_t* __restrict__ B, DevCount nbc,
                                                         const uint32_t* __restrict__ splits,
                                                         uint32_t* __restrict__ lb) {
  __shared__ uint32_t sA[MP_TILE];
  __shared__ uint32_t sB[MP_TILE];
  const uint32_t na = nac.get(), nb = nbc.get();
  const uint64_t total = (uint64_t)na + nb;
  const uint32_t d0 = blockIdx.x * MP_TILE;
  if ((uint64_t)d0 >= total) return;  // beyond the device-side counts (block-uniform)
  const uint32_t d1 = (uint32_t)min((uint64_t)d0 + MP_TILE, total);
  const uint32_t i0 = splits[blockIdx.x], i1 = splits[blockIdx.x + 1];
  const uint32_t j0 = d0 - i0, j1 = d1 - i1;
  const uint32_t la = i1 - i0, lb_ = j1 - j0;
  for (uint32_t k = threadIdx.x; k < la; k += MP_THREADS) sA[k] = A[i0 + k];
  for (uint32_t k = threadIdx.x; k < lb_; k += MP_THREADS) sB[k] = B[j0 + k];
  __syncthreads();
  const uint32_t dl = threadIdx.x * MP_ITEMS;
  if (dl >= la + lb_) return;
  uint32_t ia = merge_split(sA, la, sB, lb_, dl);
  uint32_t jb = dl - ia;
  const uint32_t steps = min((uint32_t)MP_ITEMS, la + lb_ - dl);
  for (uint32_t s = 0; s < steps; ++s) {
    bool takeA = ia < la && (jb >= lb_ || sA[ia] <= sB[jb]);
    if (takeA) {
      lb[i0 + ia] = j0 + jb;
      ++ia;
    } else {
      ++jb;
    }
  }
}

// ---------------------------------------------------------------------------
// per-group B ranges
// ---------------------------------------------------------------------------
// first p in [lo, hi] with keys[p] >= K (hi if none), searching from `hint`
__device__ inline uint32_t gallop_lower(const uint32_t* keys, uint32_t K, uint32_t hint, uint32_t lo,
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

// first p in [lo, hi] with keys[p] > K
__device__ inline uint32_t gallop_upper(const uint32_t* keys, uint32_t K, uint32_t hint, uint32_t lo,
                                        uint32_t hi) {
  if (K == 0xffffffffu) return hi;
  return gallop_lower(keys, K + 1u, hint, lo, hi);
}

// Coarse index of sorted keys: idx[i] = first position with key >= i << shift,
// for i < T (T = (key space >> shift) + 1).
// Built by one pass over the sorted keys: position p is the entry
// of every index slot i with key[p - 1] >> shift < i <= key[p] >> shift
// (slots from 0 for p = 0, up to T - 1 for p = n), so every slot is written
// exactly once. Short runs of slots are written by their lane, long ones
// (empty stretches of key space) by the whole wave.
constexpr uint32_t KI_PER = 4;  // positions per thread

__global__ __launch_bounds__(256) void k_key_index_scan(const uint32_t* __restrict__ keys, DevCount nc, int shift,
                                                        uint32_t T, uint32_t* __restrict__ idx) {
  const uint32_t n = nc.get();
  const uint32_t p0 = (blockIdx.x * blockDim.x + threadIdx.x) * KI_PER;
  const uint32_t lane = threadIdx.x & 63u;
  // keys p0 - 1 .. p0 + KI_PER - 1 (one 16-B load when all are present)
  uint32_t k[KI_PER];
  uint32_t prev = 0u;
  if (p0 + KI_PER <= n) {
    const uint4 v = *reinterpret_cast<const uint4*>(keys + p0);
    k[0] = v.x;
    k[1] = v.y;
    k[2] = v.z;
    k[3] = v.w;
  } else {
#pragma unroll
    for (uint32_t q = 0; q < KI_PER; ++q) k[q] = p0 + q < n ? keys[p0 + q] : 0u;
  }
  if (p0 > 0 && p0 <= n) prev = keys[p0 - 1];
#pragma unroll
  for (uint32_t q = 0; q < KI_PER; ++q) {
    const uint32_t p = p0 + q;
    uint32_t lo = 0u, hi = 0u;  // slots [lo, hi) get p
    if (p <= n) {
      lo = p == 0 ? 0u : (prev >> shift) + 1u;
      hi = p == n ? T : min((k[q] >> shift) + 1u, T);
      if (hi < lo) hi = lo;
    }
    prev = k[q];
    constexpr uint32_t SHORT = 4;
    const bool is_long = hi - lo > SHORT;
    if (!is_long)
      for (uint32_t i = lo; i < hi; ++i) idx[i] = p;
    uint64_t longs = __ballot(is_long);
    while (longs) {
      const int l = __builtin_ctzll(longs);
      longs &= longs - 1ull;
      const uint32_t L0 = (uint32_t)__shfl((int)lo, l), L1 = (uint32_t)__shfl((int)hi, l);
      const uint32_t P = (uint32_t)__shfl((int)p, l);
      for (uint32_t i = L0 + lane; i < L1; i += 64u) idx[i] = P;
    }
  }
}

// First position in [lo, hi) whose key is >= K (hi if none), searched only
// between the two index entries that bracket K.
__device__ inline uint32_t index_lower(const uint32_t* keys, const uint32_t* idx, int shift, uint32_t T,
                                       uint64_t K, uint32_t lo, uint32_t hi) {
  const uint64_t i = K >> shift;
  if (i + 1 >= T) return hi;
  uint32_t l = max(lo, idx[i]), r = min(hi, idx[i + 1]);
  if (l > r) l = r;
  while (l < r) {
    const uint32_t mid = l + ((r - l) >> 1);
    if (keys[mid] < (uint32_t)K) l = mid + 1; else r = mid;
  }
  return l;
}

// index_lower of two keys at once: the two searches advance in lockstep, so
// each step's two loads are in flight together (keys[0] stands in for a
// finished search: every key buffer holds at least one entry)
__device__ inline void index_lower2(const uint32_t* keys, const uint32_t* idx, int shift, uint32_t T,
                                    uint64_t K1, uint64_t K2, uint32_t lo, uint32_t hi, uint32_t& r1,
                                    uint32_t& r2) {
  auto bracket = [&](uint64_t K, uint32_t& l, uint32_t& r) {
    const uint64_t i = K >> shift;
    if (i + 1 >= T) {
      l = r = hi;
      return;
    }
    l = max(lo, idx[i]);
    r = min(hi, idx[i + 1]);
    if (l > r) l = r;
  };
  uint32_t l1, h1, l2, h2;
  bracket(K1, l1, h1);
  bracket(K2, l2, h2);
  while (l1 < h1 || l2 < h2) {
    const bool a1 = l1 < h1, a2 = l2 < h2;
    const uint32_t m1 = l1 + ((h1 - l1) >> 1), m2 = l2 + ((h2 - l2) >> 1);
    const uint32_t k1 = keys[a1 ? m1 : 0u], k2 = keys[a2 ? m2 : 0u];
    if (a1) {
      if (k1 < (uint32_t)K1) l1 = m1 + 1; else h1 = m1;
    }
    if (a2) {
      if (k2 < (uint32_t)K2) l2 = m2 + 1; else h2 = m2;
    }
  }
  r1 = l1;
  r2 = l2;
}

// One thread per group of GROUP consecutive sorted A entries; the group's
// keys are staged in LDS (a per-thread row, read with runtime indices).
constexpr int RG_STRIDE = GROUP + 1;  // padded row: no LDS bank conflicts
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keysA, DevCount nac,
                                                const uint32_t* __restrict__ kidx, int kshift, uint32_t kT,
                                                const uint32_t* __restrict__ keysB,
                                                const uint32_t* __restrict__ zstartB,
                                                const int32_t* __restrict__ zmarg,
                                                const double* __restrict__ zdelta, Geom g,
                                                GroupRanges* __restrict__ out) {
  __shared__ uint32_t s_keys[256 * RG_STRIDE];
  const uint32_t na = nac.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  uint32_t grp = blockIdx.x * blockDim.x + threadIdx.x;
  if (grp >= ngroups) return;
  const uint32_t p0 = grp * GROUP;
  const uint32_t cnt = min((uint32_t)GROUP, na - p0);
  uint32_t* k = s_keys + threadIdx.x * RG_STRIDE;  // this thread's row only
  if (cnt == (uint32_t)GROUP) {
    // the group's keys in four 16-B loads (p0 is a multiple of 16)
    const uint4* k4 = reinterpret_cast<const uint4*>(keysA + p0);
    uint4 v[GROUP / 4];
#pragma unroll
    for (int r = 0; r < GROUP / 4; ++r) v[r] = k4[r];
#pragma unroll
    for (int r = 0; r < GROUP / 4; ++r) {
      k[4 * r] = v[r].x;
      k[4 * r + 1] = v[r].y;
      k[4 * r + 2] = v[r].z;
      k[4 * r + 3] = v[r].w;
    }
  } else {
    for (uint32_t q = 0; q < cnt; ++q) k[q] = keysA[p0 + q];
  }
  RangeList L;
  L.clear();
  const int64_t nbins = g.nbins;
  uint32_t q = 0;
  while (q < cnt) {
    const int32_t z = key_zone(g, k[q]);
    uint32_t qe = q;
    while (qe + 1 < cnt && key_zone(g, k[qe + 1]) == z) ++qe;
    const uint32_t zs = zstartB[z], ze = zstartB[z + 1];
    const int64_t bf = key_bin(g, k[q]), bl = key_bin(g, k[qe]);
    const int32_t m = zmarg[z];
    int64_t lo = bf - m, hi = bl + m;
    // sub-bin positions of the window's edges (searched only when B's keys
    // are sorted on their sub-bin bits as well)
    const uint32_t cell_top = (1u << g.fb) - 1u;
    uint32_t flo = 0u, fhi = cell_top;
    if (m >= 0) {
      // the window from the bin edges of the segment's first and last
      // sources: bf * width is exact (width = 360 / 2^rb), bin_of is
      // monotone, and the half-width D is padded beyond every rounding, so
      // every B within r of a source of bins bf..bl lies in bins lo..hi
      // (the sub-bin fractions of the sources in the first and last bins
      // narrow the edges to 2^-fb bin; width and its fractions are exact)
      const double width = g.ra_width;
      const double fw = width / (double)(1u << g.fb);
      uint32_t fmin = (1u << g.fb) - 1u, fmax = 0u;
      for (uint32_t u = q; u <= qe; ++u) {
        const int64_t bu = key_bin(g, k[u]);
        if (bu == bf) fmin = min(fmin, key_frac(g, k[u]));
        if (bu == bl) fmax = max(fmax, key_frac(g, k[u]));
      }
      const double D = zdelta[z];
      const double x = g.ra0 + ((double)bf * width + (double)fmin * fw) - D;
      const double y = g.ra0 + ((double)bl * width + (double)(fmax + 1u) * fw) + D;
      if (g.full_ra) {
        lo = x >= 0.0 ? (int64_t)bin_of(g, x) : (int64_t)bin_of(g, x + 360.0) - nbins;
        hi = y < 360.0 ? (int64_t)bin_of(g, y) : (int64_t)bin_of(g, y - 360.0) + nbins;
      } else {
        // a partial frame holds every source and spans less than 180 deg
        // of RA, so no pair crosses its RA edges: clamp, never wrap
        lo = (int64_t)bin_of(g, x);
        hi = (int64_t)bin_of(g, y);
      }
      if (g.frac_sorted) {
        // the key is monotone in RA within a zone, so every B entry of RA in
        // [x, y] lies between the keys of the two edges (taken in the bin
        // each edge falls in, after the wrap at the seam)
        const double xe = (g.full_ra && x < 0.0) ? x + 360.0 : x;
        const double ye = (g.full_ra && y >= 360.0) ? y - 360.0 : y;
        flo = frac_of(g, xe, bin_of(g, xe));
        fhi = frac_of(g, ye, bin_of(g, ye));
      }
    }
    if (m < 0 || hi - lo + 1 >= nbins) {
      L.add(zs, ze);
    } else if (zs < ze) {
      auto lower = [&](uint64_t K) { return index_lower(keysB, kidx, kshift, kT, K, zs, ze); };
      // (the end of a cell: its last key + 1 = the first key of the next;
      // with sorted sub-bin bits, the edge's own key + 1)
      const uint64_t cell = 1ull << g.fb;
      uint32_t s, e;
      index_lower2(keysB, kidx, kshift, kT,
                   (uint64_t)make_key(g, z, (uint32_t)(lo < 0 ? 0 : lo)) + (lo < 0 ? 0u : flo),
                   (uint64_t)make_key(g, z, (uint32_t)(hi > nbins - 1 ? nbins - 1 : hi)) +
                       (hi > nbins - 1 ? cell : (uint64_t)fhi + 1u),
                   zs, ze, s, e);
      if (hi > nbins - 1) {  // window passes RA 360: low bins of the zone
        uint32_t e2 = lower((uint64_t)make_key(g, z, (uint32_t)(hi - nbins)) + (uint64_t)fhi + 1u);
        L.add(zs, e2);
      }
      L.add(s, e);
      if (lo < 0) {  // window passes RA 0: high bins of the zone
        uint32_t s2 = lower((uint64_t)make_key(g, z, (uint32_t)(nbins + lo)) + flo);
        L.add(s2, ze);
      }
    }
    q = qe + 1;
  }
  GroupRanges R;
#pragma unroll
  for (int t = 0; t < MAXR; ++t) {
    R.start[t] = t < L.n ? L.s[t] : 0u;
    R.end[t] = t < L.n ? L.e[t] : 0u;
  }
  R.count = (uint32_t)L.n;
  R.pad_[0] = R.pad_[1] = R.pad_[2] = 0u;
  out[grp] = R;
}

// largest error radius (order-preserving code of a non-negative double is its
// bit pattern); bit 8 of err flags a negative or non-finite value
__global__ __launch_bounds__(256) void k_err_max(const double* __restrict__ err, uint32_t n,
                                                 unsigned long long* __restrict__ out, Counters* cnt) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c = 0ull;
  if (i < n) {
    const double e = err[i];
    if (e >= 0.0 && e <= 1.0e300) c = (unsigned long long)__double_as_longlong(e);
    else atomicOr(&cnt->err, 8u);
  }
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(c, off);
    c = o > c ? o : c;
  }
  if ((threadIdx.x & 63) == 0 && c) atomicMax(out, c);
}

// ---------------------------------------------------------------------------
// paper-scheme emulation
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hp_keygen(const double* __restrict__ ra,
                                                   const double* __restrict__ dec, uint32_t n, int order,
                                                   double R, uint32_t err_bit, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals,
                                                   unsigned long long* __restrict__ count, Counters* cnt) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t px[5];
  int m = 0;
  if (i < n) {
    const double a = ra[i], d = dec[i];
    if (valid_pos(a, d)) m = hp_quad(order, a, d, R, px);
    else atomicOr(&cnt->err, err_bit);
  }
  // wave prefix of the entry counts, one atomic per wave
  const uint32_t lane = lane_id();
  uint32_t x = (uint32_t)m;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= (uint32_t)off) x += y;
  }
  const uint32_t total = __shfl(x, 63);
  unsigned long long base = 0;
  if (lane == 63 && total) base = atomicAdd(count, (unsigned long long)total);
  base = __shfl(base, 63);
  const unsigned long long pos = base + x - (uint32_t)m;
  for (int k = 0; k < m; ++k) {
    keys[pos + k] = px[k];
    vals[pos + k] = i;
  }
}

__global__ __launch_bounds__(256) void k_radec_gather(const uint32_t* __restrict__ vals, DevCount nc,
                                                      const double* __restrict__ ra,
                                                      const double* __restrict__ dec,
                                                      double2* __restrict__ radec) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nc.get()) return;
  const uint32_t i = vals[p] & IDX_MASK;
  radec[p] = make_double2(ra[i], dec[i]);
}

__global__ __launch_bounds__(256) void k_equal_ranges(const uint32_t* __restrict__ keysA, DevCount nac,
                                                      const uint32_t* __restrict__ lb,
                                                      const uint32_t* __restrict__ keysB, DevCount nbc,
                                                      GroupRanges* __restrict__ out) {
  const uint32_t na = nac.get(), nb = nbc.get();
  const uint32_t ngroups = (na + GROUP - 1) / GROUP;
  const uint32_t grp = blockIdx.x * blockDim.x + threadIdx.x;
  if (grp >= ngroups) return;
  const uint32_t p0 = grp * GROUP, cnt = min((uint32_t)GROUP, na - p0);
  RangeList L;
  L.clear();
  uint32_t q = 0;
  while (q < cnt) {
    const uint32_t k = keysA[p0 + q];
    uint32_t qe = q;
    while (qe + 1 < cnt && keysA[p0 + qe + 1] == k) ++qe;
    const uint32_t s = lb[p0 + q];  // first B key >= k
    const uint32_t e = gallop_upper(keysB, k, s, s, nb);
    L.add(s, e);
    q = qe + 1;
  }
  GroupRanges R;
#pragma unroll
  for (int t = 0; t < MAXR; ++t) {
    R.start[t] = t < L.n ? L.s[t] : 0u;
    R.end[t] = t < L.n ? L.e[t] : 0u;
  }
  R.count = (uint32_t)L.n;
  R.pad_[0] = R.pad_[1] = R.pad_[2] = 0u;
  out[grp] = R;
}

// ---------------------------------------------------------------------------
// ordering of an output pair list by (a, b)
// ---------------------------------------------------------------------------
__global__ void k_pairs_keys(const uint2* __restrict__ p, uint32_t n, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ vals) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    keys[i] = p[i].y;
    vals[i] = i;
  }
}

__global__ void k_pairs_rekey(const uint2* __restrict__ p, const uint32_t* __restrict__ vals, uint32_t n,
                              uint32_t* __restrict__ keys) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = p[vals[i]].x;
}

__global__ void k_pairs_permute(const uint2* __restrict__ p, const double* __restrict__ sep,
                                const uint32_t* __restrict__ vals, uint32_t n, uint2* __restrict__ tp,
                                double* __restrict__ ts) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const uint32_t j = vals[i];
    tp[i] = p[j];
    if (sep) ts[i] = sep[j];
  }
}

// ---------------------------------------------------------------------------
// data footprint (Dec and RA extent of valid sources) for the geometry frame
// ---------------------------------------------------------------------------
__device__ inline unsigned long long ord_code(double v) {  // v >= 0
  return (unsigned long long)__double_as_longlong(v);
}

// Block-wide max of e[4] into cnt->ext: atomically (several blocks), or
// stored (one block; then also mirrored to msg[0..3] in host memory,
// followed by msg[4] = seq once the four values are visible there).
__device__ inline void ext_reduce(unsigned long long e[4], Counters* cnt, bool block_level,
                                  unsigned long long* msg = nullptr, unsigned long long seq = 0ull) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
    for (int d = 32; d > 0; d >>= 1) {
      const unsigned long long o = __shfl_xor(e[k], d);
      e[k] = o > e[k] ? o : e[k];
    }
  __shared__ unsigned long long s_e[16][4];  // up to 16 waves
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0)
    for (int k = 0; k < 4; ++k) s_e[w][k] = e[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m[4];
    for (int k = 0; k < 4; ++k) {
      m[k] = 0ull;
      for (uint32_t u = 0; u < (blockDim.x >> 6); ++u) m[k] = s_e[u][k] > m[k] ? s_e[u][k] : m[k];
    }
    if (block_level) {
      for (int k = 0; k < 4; ++k) atomicMax(&cnt->ext[k], m[k]);
    } else {
      for (int k = 0; k < 4; ++k) cnt->ext[k] = m[k];
      if (msg) {
        for (int k = 0; k < 4; ++k) msg[k] = m[k];
        __threadfence_system();
        msg[4] = seq;
      }
    }
  }
}

__device__ inline void ext_add(unsigned long long e[4], double a, double d) {
  if (!valid_pos(a, d)) return;
  const unsigned long long cd = ord_code(d + 90.0), ca = ord_code(a);
  e[0] = ~cd > e[0] ? ~cd : e[0];
  e[1] = cd > e[1] ? cd : e[1];
  e[2] = ~ca > e[2] ? ~ca : e[2];
  e[3] = ca > e[3] ? ca : e[3];
}

// One block of 1024 threads: a sample of up to 2 x 4096 sources, 64 runs
// of 64 consecutive sources per catalogue, evenly spaced (few pages, so few
// address translations); every load is issued before the first use.
__device__ inline uint32_t sample_index(uint32_t run, uint32_t lane, uint32_t n) {
  if (n <= 64u) return lane % n;
  const uint32_t start = (uint32_t)(((uint64_t)run * n) / 64u);
  return min(start, n - 64u) + lane;
}

__global__ __launch_bounds__(1024) void k_extent_sample(const double* __restrict__ ra1,
                                                        const double* __restrict__ dec1, uint32_t n1,
                                                        const double* __restrict__ ra2,
                                                        const double* __restrict__ dec2, uint32_t n2, Counters* cnt,
                                                        unsigned long long* msg, unsigned long long seq) {
  constexpr int PER = 4;  // runs per wave and catalogue (16 waves x 4 = 64 runs)
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  double a[2 * PER], d[2 * PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint32_t run = w + 16u * (uint32_t)j;
    const uint32_t i1 = n1 ? sample_index(run, lane, n1) : 0u, i2 = n2 ? sample_index(run, lane, n2) : 0u;
    a[j] = n1 ? ra1[i1] : -1.0;
    d[j] = n1 ? dec1[i1] : 0.0;
    a[PER + j] = n2 ? ra2[i2] : -1.0;
    d[PER + j] = n2 ? dec2[i2] : 0.0;
  }
  unsigned long long e[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
  for (int j = 0; j < 2 * PER; ++j) ext_add(e, a[j], d[j]);
  ext_reduce(e, cnt, false, msg, seq);
}

// Every source; one atomic per value and block.
__global__ __launch_bounds__(256) void k_extent(const double* __restrict__ ra, const double* __restrict__ dec,
                                                uint32_t n, Counters* cnt) {
  unsigned long long e[4] = {0ull, 0ull, 0ull, 0ull};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    ext_add(e, ra[i], dec[i]);
  ext_reduce(e, cnt, true);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_hp_keygen(const double* ra, const double* dec, uint32_t n, int order, double R, uint32_t err_bit,
                      uint32_t* keys, uint32_t* vals, unsigned long long* count, Counters* cnt, hipStream_t s) {
  if (n == 0) return;
  k_hp_keygen<<<cdiv(n, 256), 256, 0, s>>>(ra, dec, n, order, R, err_bit, keys, vals, count, cnt);
}

void launch_radec_gather(const uint32_t* vals, const DevCount& n, const double* ra, const double* dec,
                         double2* radec, hipStream_t s) {
  if (n.cap == 0) return;
  k_radec_gather<<<cdiv(n.cap, 256), 256, 0, s>>>(vals, n, ra, dec, radec);
}

void launch_equal_ranges(const uint32_t* keysA, const DevCount& na, const uint32_t* lb, const uint32_t* keysB,
                         const DevCount& nb, GroupRanges* out, hipStream_t s) {
  const uint32_t ng = cdiv(na.cap, GROUP);
  if (ng == 0) return;
  k_equal_ranges<<<cdiv(ng, 256), 256, 0, s>>>(keysA, na, lb, keysB, nb, out);
}

void launch_err_max(const double* err, uint32_t n, unsigned long long* out_code, Counters* cnt,
                    hipStream_t s) {
  if (n == 0) return;
  k_err_max<<<cdiv(n, 256), 256, 0, s>>>(err, n, out_code, cnt);
}

void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return;
  uint32_t blocks = (uint32_t)std::min<size_t>((n + 255) / 256, 4096);
  k_fill_u32<<<blocks, 256, 0, s>>>(p, v, n);
}

void launch_zero_counters(Counters* c, hipStream_t s) { k_zero_counters<<<1, 64, 0, s>>>(c); }

void launch_keygen(const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
                   uint32_t err_bit, uint32_t* keys, uint32_t* vals, Counters* cnt, hipStream_t s,
                   double2* radec, const KeygenHist* kh, bool iota_vals) {
  if (n == 0) return;
  uint32_t* hist = nullptr;
  uint32_t tiles = 0, full = 0;
  int shift = 0;
  if (kh) {
    tiles = cdiv(kh->cap, RS_TILE);
    full = n / RS_TILE;
    shift = kh->shift;
    // (each of those tiles' counts is stored whole by its block: no clearing)
    hist = full ? kh->counts : nullptr;
  }
  k_keygen<<<std::max<uint32_t>(1, cdiv(n, KG_TILE)), KG_THREADS, 0, s>>>(
      ra, dec, n, g, halo ? 1 : 0, err_bit, keys, vals, cnt, radec, hist, tiles, shift,
      full, iota_vals ? 1 : 0);
}

size_t sort_counts_len(uint32_t n) { return (size_t)RS_BINS * std::max<uint32_t>(1, cdiv(n, RS_TILE)); }
size_t sort_digit_totals_len(uint32_t n) { (void)n; return RS_BINS; }

int radix_passes(int key_bits, int lo_bit) { return (key_bits - lo_bit + 7) / 8; }

uint32_t keygen_hist_tiles(uint32_t n) { return n / RS_TILE; }

// blocks of the persistent scatter: two per CU (as many as its LDS allows)
static uint32_t scatter_blocks() {
  static const uint32_t v = [] {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
      (void)hipGetLastError();
      cus = 256;
    }
    return 2u * (uint32_t)cus;
  }();
  return v;
}

void radix_sort(uint32_t* keys, uint32_t* vals, const DevCount& cnt, int key_bits, const SortScratch& sc,
                hipStream_t s, bool from_alt, int lo_bit, uint32_t hist_done, uint32_t iota) {
  const uint32_t n = cnt.cap;  // grids cover the capacity; kernels read the count
  const int passes = radix_passes(key_bits, lo_bit);
  uint32_t *kin = keys, *vin = vals, *kout = sc.keys_alt, *vout = sc.vals_alt;
  if (from_alt) {
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (n > 1) {
    const uint32_t ntiles = cdiv(n, RS_TILE);
    for (int p = 0; p < passes; ++p) {
      const int shift = lo_bit + 8 * p;
      // the first pass's counts of tiles below hist_done came from the keygen
      const uint32_t h0 = p == 0 ? std::min(hist_done, ntiles) : 0u;
      if (h0 < ntiles) k_radix_hist<<<ntiles - h0, RS_THREADS, 0, s>>>(kin, cnt, shift, sc.counts, ntiles, h0);
      k_scan_digits<<<RS_BINS, RS_THREADS, 0, s>>>(sc.counts, ntiles, sc.digit_totals);
      k_radix_scatter<<<std::min<uint32_t>(ntiles, scatter_blocks()), SC_THREADS, 0, s>>>(
          kin, vin, kout, vout, cnt, shift, sc.counts, sc.digit_totals, ntiles, p == 0 ? iota : 0u);
      std::swap(kin, kout);
      std::swap(vin, vout);
    }
  }
  if (kin != keys && n > 0) k_copy_pairs<<<cdiv(n, 256), 256, 0, s>>>(kin, vin, keys, vals, cnt);
}

void sort_pairs(uint2* pairs, double* sep, uint32_t n, int bits_a, int bits_b, uint32_t* keys, uint32_t* vals,
                uint2* tmp_pairs, double* tmp_sep, const SortScratch& sc, hipStream_t s) {
  if (n <= 1) return;
  const DevCount cnt{n, n, nullptr};
  // stable by b, then stable by a: (a, b) order
  k_pairs_keys<<<cdiv(n, 256), 256, 0, s>>>(pairs, n, keys, vals);
  radix_sort(keys, vals, cnt, bits_b, sc, s);
  k_pairs_rekey<<<cdiv(n, 256), 256, 0, s>>>(pairs, vals, n, keys);
  radix_sort(keys, vals, cnt, bits_a, sc, s);
  k_pairs_permute<<<cdiv(n, 256), 256, 0, s>>>(pairs, sep, vals, n, tmp_pairs, tmp_sep);
  (void)hipMemcpyAsync(pairs, tmp_pairs, (size_t)n * sizeof(uint2), hipMemcpyDeviceToDevice, s);
  if (sep) (void)hipMemcpyAsync(sep, tmp_sep, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
}

void launch_extent_sample(const double* ra1, const double* dec1, uint32_t n1, const double* ra2, const double* dec2,
                          uint32_t n2, Counters* cnt, unsigned long long* msg, unsigned long long seq,
                          hipStream_t s) {
  k_extent_sample<<<1, 1024, 0, s>>>(ra1, dec1, n1, ra2, dec2, n2, cnt, msg, seq);
}

void launch_extent(const double* ra, const double* dec, uint32_t n, Counters* cnt, hipStream_t s) {
  if (n == 0) return;
  k_extent<<<std::min<uint32_t>(1024, cdiv(n, 256 * 64)), 256, 0, s>>>(ra, dec, n, cnt);
}

void launch_zone_tables(const Geom& g, int32_t* zmarg, double* zdelta, hipStream_t s) {
  k_zone_tables<<<cdiv((uint32_t)g.nz, 256), 256, 0, s>>>(g, zmarg, zdelta);
}

void launch_zone_starts_index(const uint32_t* idx, int shift, uint32_t T, const DevCount& n, const Geom& g,
                              uint32_t* zstart, hipStream_t s, int32_t* zmarg, double* zdelta) {
  k_zone_starts_index<<<cdiv((uint32_t)g.nz + 1, 256), 256, 0, s>>>(idx, shift, T, n, g, zstart, zmarg, zdelta);
}

void launch_zone_starts(const uint32_t* keys, const DevCount& n, const Geom& g, uint32_t* zstart,
                        hipStream_t s) {
  k_zone_starts<<<cdiv((uint32_t)g.nz + 1, 256), 256, 0, s>>>(keys, n, g, zstart);
}

void launch_layout64(const uint32_t* vals, const DevCount& n, const double* ra, const double* dec,
                     Rec64* rec, hipStream_t s, const double2* il) {
  if (n.cap == 0) return;
  k_layout64<<<cdiv(n.cap, 256), 256, 0, s>>>(vals, n, ra, dec, il, rec);
}

void launch_layout32(const uint32_t* vals, const DevCount& n, const double* ra, const double* dec,
                     CellRec32* rec, double2* radec, hipStream_t s, const double2* il) {
  if (n.cap == 0) return;
  k_layout32<<<cdiv(n.cap, 256), 256, 0, s>>>(vals, n, ra, dec, il, rec, radec);
}

size_t merge_splits_len(uint64_t na_cap, uint64_t nb_cap) { return (size_t)cdiv(na_cap + nb_cap, MP_TILE) + 1; }

void launch_merge_lb(const uint32_t* keysA, const DevCount& na, const uint32_t* keysB,
                     const DevCount& nb, uint32_t* splits, uint32_t* lb, hipStream_t s) {
  if (na.cap == 0) return;
  const uint32_t blocks = cdiv((uint64_t)na.cap + nb.cap, MP_TILE);
  k_merge_splits<<<cdiv(blocks + 1, 256), 256, 0, s>>>(keysA, na, keysB, nb, blocks + 1, splits);
  k_merge_lb<<<blocks, MP_THREADS, 0, s>>>(keysA, na, keysB, nb, splits, lb);
}

void launch_key_index(const uint32_t* keys, const DevCount& n, int shift, uint32_t T, uint32_t* idx,
                      hipStream_t s) {
  k_key_index_scan<<<cdiv(cdiv((uint64_t)n.cap + 1, KI_PER), 256), 256, 0, s>>>(keys, n, shift, T, idx);
}

void launch_ranges(const uint32_t* keysA, const DevCount& na, const uint32_t* kidx, int kshift, uint32_t kT,
                   const uint32_t* keysB, const uint32_t* zstartB, const int32_t* zmarg, const double* zdelta,
                   const Geom& g, GroupRanges* out, hipStream_t s) {
  uint32_t ngroups = cdiv(na.cap, GROUP);
  if (ngroups == 0) return;
  k_ranges<<<cdiv(ngroups, 256), 256, 0, s>>>(keysA, na, kidx, kshift, kT, keysB, zstartB, zmarg, zdelta, g,
                                                 out);
}

}  // namespace hlc
