// hlc_kernels.hpp -- host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hlc_device.hpp"

namespace hlc {

// ---- partition.hip ---------------------------------------------------------
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void launch_zero_counters(Counters* c, hipStream_t s);
struct SortScratch {
  uint32_t* keys_alt;
  uint32_t* vals_alt;
  uint32_t* counts;     // 256 * ntiles
  uint32_t* digit_totals; // per-digit totals of one pass
};

// The first radix pass's per-tile digit counts, filled by the keygen for
// the tiles it alone writes (the sort's scratch counts of an entry capacity
// cap, digit shift of the first pass).
struct KeygenHist {
  uint32_t* counts;
  uint32_t cap;
  int shift;
};
// keys/vals of n sources: one entry per source, plus the Dec-halo copies
// appended after n when `halo` is set (with iota_vals, the value of source
// i, i itself, is left to the sort's first pass); with radec also each
// source's (ra, dec) as one 16-B record in input order, the per-source
// record that the layouts, the filter (a side read in place) and the
// certification read
void launch_keygen(const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
                   uint32_t err_bit, uint32_t* keys, uint32_t* vals, Counters* cnt, hipStream_t s,
                   double2* radec = nullptr, const KeygenHist* kh = nullptr, bool iota_vals = false);
// tiles of the first pass whose counts a keygen of n sources fills
uint32_t keygen_hist_tiles(uint32_t n);

size_t sort_counts_len(uint32_t n);
size_t sort_digit_totals_len(uint32_t n);
// Stable LSD radix sort of (keys, vals), ascending, by key bits
// [lo_bit, key_bits) (lower bits ride along unsorted); the result is in
// (keys, vals). With from_alt the input is in the scratch pair instead:
// callers that write their input there when radix_passes(...) is odd spare
// the final copy.
int radix_passes(int key_bits, int lo_bit = 0);
// n output pairs (and their separations, if sep) ordered by (a, b); keys,
// vals, tmp_pairs, tmp_sep hold n entries each
void sort_pairs(uint2* pairs, double* sep, uint32_t n, int bits_a, int bits_b, uint32_t* keys, uint32_t* vals,
                uint2* tmp_pairs, double* tmp_sep, const SortScratch& sc, hipStream_t s);
// hist_done: tiles whose first-pass counts are already in sc.counts (keygen);
// iota: entries below it take their position as value in the first pass
// (their values are not read: with iota_vals the keygen does not write them;
// at least one pass must run)
void radix_sort(uint32_t* keys, uint32_t* vals, const DevCount& n, int key_bits, const SortScratch& sc,
                hipStream_t s, bool from_alt = false, int lo_bit = 0, uint32_t hist_done = 0,
                uint32_t iota = 0);

// footprint of the valid sources into Counters::ext (max-combined): a
// sample of at most 2 x 4096 sources (overwrites; also written to msg[0..3]
// in mapped host memory, then msg[4] = seq), or every source (combines)
void launch_extent_sample(const double* ra1, const double* dec1, uint32_t n1, const double* ra2, const double* dec2,
                          uint32_t n2, Counters* cnt, unsigned long long* msg, unsigned long long seq,
                          hipStream_t s);
void launch_extent(const double* ra, const double* dec, uint32_t n, Counters* cnt, hipStream_t s);
void launch_zone_tables(const Geom& g, int32_t* zmarg, double* zdelta, hipStream_t s);
void launch_zone_starts(const uint32_t* keys, const DevCount& n, const Geom& g, uint32_t* zstart,
                        hipStream_t s);
// the same read from the key index (requires rb + fb >= shift: every zone's
// first key is then a multiple of the index step); with zmarg, also the zone
// tables of launch_zone_tables
void launch_zone_starts_index(const uint32_t* idx, int shift, uint32_t T, const DevCount& n, const Geom& g,
                              uint32_t* zstart, hipStream_t s, int32_t* zmarg = nullptr,
                              double* zdelta = nullptr);
// sorted working records of a side: each entry's source position read from
// il (the keygen's (ra, dec) records) when given, else from ra and dec
void launch_layout64(const uint32_t* vals, const DevCount& n, const double* ra, const double* dec,
                     Rec64* rec, hipStream_t s, const double2* il = nullptr);
// (and the sorted (ra, dec) when radec is not null)
void launch_layout32(const uint32_t* vals, const DevCount& n, const double* ra, const double* dec,
                     CellRec32* rec, double2* radec, hipStream_t s, const double2* il = nullptr);
// lb[i] = number of B keys below keysA[i]; splits: merge_splits_len words of scratch
size_t merge_splits_len(uint64_t na_cap, uint64_t nb_cap);
void launch_merge_lb(const uint32_t* keysA, const DevCount& na, const uint32_t* keysB,
                     const DevCount& nb, uint32_t* splits, uint32_t* lb, hipStream_t s);
// idx[i] = first position of the sorted keys with key >= i << shift, i < T
void launch_key_index(const uint32_t* keys, const DevCount& n, int shift, uint32_t T, uint32_t* idx,
                      hipStream_t s);
void launch_ranges(const uint32_t* keysA, const DevCount& na, const uint32_t* kidx, int kshift, uint32_t kT,
                   const uint32_t* keysB, const uint32_t* zstartB, const int32_t* zmarg, const double* zdelta,
                   const Geom& g, GroupRanges* out, hipStream_t s);

// ---- match.hip -------------------------------------------------------------
// Output allocation. A single counter bumped by every wave serialises at the
// memory side (device-scope atomics on one address: a few ns each), so the
// filter appends its candidates to NREG striped staging regions (region =
// wave index mod NREG, counters 256 B apart). The certification of a single
// call writes its pairs straight into the caller's buffer, one atomic on the
// pair count per block and round of 1,024 candidates (OutArgs::direct); the
// batched form and the paper-scheme emulation stage pairs in regions too, and
// a compaction kernel packs them into the caller's buffer in region order.
constexpr int NREG = 256;
constexpr int REG_STRIDE = 32;  // u64 slots between two region counters

// A staged filter candidate.
//   FP64 form: everything the certification needs of the A entry travels
//     with it, so the certification reads nothing of A: (u0, u1, u2) is A's
//     FP64 unit vector, ia A's original index (paper-scheme emulation: A's
//     sorted position), b B's sorted position.
//   FP32 form: (u0, u1) is A's (ra, dec) when the filter has it (A read in
//     place, or A's (ra, dec) sorted), else NaN; ia and b are A's and B's
//     original indices, bpos B's sorted position; the certification reads
//     B's (ra, dec) at bpos when they are sorted (the candidates of one wave
//     lie in a few B windows, so those reads share cache lines), else by b.
struct Cand {
  double u0, u1;
  union {
    double u2;      // FP64 form
    uint32_t bpos;  // FP32 form
  };
  uint32_t ia, b;
};

struct Regions {
  unsigned long long* fill;     // NREG * REG_STRIDE; fill[k * REG_STRIDE] = pairs sent to region k
  unsigned long long* cfill;    // NREG * REG_STRIDE; candidates sent to region k
  uint2* pairs;                 // NREG * S staging (nullptr when S = 0: pairs written directly)
  double* sep;                  // NREG * S staging, or nullptr
  unsigned long long S;         // pair slots per region
  Cand* cand;                   // NREG * Sc staged candidates, or nullptr
  unsigned long long Sc;        // candidate slots per region (0: candidates are only counted)
  unsigned long long* cpre;     // NREG + 1: exclusive prefix of the staged candidate counts
};

struct OutArgs {
  uint2* pairs;                 // caller buffer (a, b)
  double* sep;                  // caller buffer or nullptr
  unsigned long long cap;       // capacity in pairs
  uint2* band;                  // band list (original indices, B halo bit cleared)
  uint32_t* band_job;           // batched form: job of each band entry (else nullptr)
  unsigned long long band_cap;
  Counters* cnt;
  Regions reg;
  int direct;  // certified pairs straight into pairs/sep (block-aggregated counter), not through regions
};

__device__ inline uint32_t wave_region() {
  return ((blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6)) & (NREG - 1);
}

// Pairs of the lanes with `in` set, appended to this wave's region with one
// atomic.
__device__ inline void emit_wave(bool in, uint32_t ia, uint32_t ib, double sep, const OutArgs& o) {
  const uint64_t m = __ballot(in);
  if (m == 0) return;
  const uint32_t k = wave_region();
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(&o.reg.fill[k * REG_STRIDE], (unsigned long long)__popcll(m));
  base = __shfl(base, (int)leader);
  if (in) {
    const unsigned long long slot = base + rank_in(m);
    if (slot < o.reg.S) {
      const unsigned long long at = (unsigned long long)k * o.reg.S + slot;
      o.reg.pairs[at] = make_uint2(ia, ib);
      if (o.reg.sep) o.reg.sep[at] = sep;
    }
  }
}

// One pair from one thread (rare paths: band certification).
__device__ inline void emit_one(uint32_t ia, uint32_t ib, double sep, const OutArgs& o) {
  if (o.direct) {
    const unsigned long long slot = atomicAdd(&o.cnt->n_pairs, 1ull);
    if (slot < o.cap) {
      o.pairs[slot] = make_uint2(ia, ib);
      if (o.sep) o.sep[slot] = sep;
    }
    return;
  }
  const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) & (NREG - 1);
  const unsigned long long slot = atomicAdd(&o.reg.fill[k * REG_STRIDE], 1ull);
  if (slot < o.reg.S) {
    const unsigned long long at = (unsigned long long)k * o.reg.S + slot;
    o.reg.pairs[at] = make_uint2(ia, ib);
    if (o.reg.sep) o.reg.sep[at] = sep;
  }
}

__device__ inline void count_candidates(uint32_t qn, const OutArgs& o) {
  if (lane_id() == 0) atomicAdd(&o.reg.cfill[wave_region() * REG_STRIDE], (unsigned long long)qn);
}

struct MatchArgs {
  const GroupRanges* ranges;
  DevCount na;
  // FP64 form
  const Rec64* recA64;
  const Rec64* recB64;
  double t_lo64, t_hi64;        // chord^2: certain in / candidate
  // FP32 form: sorted cell records, and the FP64 (ra, dec) of each source by
  // original index (certification; null when A is read in place, its
  // candidates then carry A's (ra, dec), or when the side has them sorted)
  const CellRec32* recA32;
  const CellRec32* recB32;
  const double2* srcradA;
  const double2* srcradB;
  float c_r32;                  // chord of r, rounded up to FP32
  // the FP64 (ra, dec) of every sorted entry, or null: FP32 certification in
  // the sorted layout, and the paper-scheme emulation
  const double2* radecA;
  const double2* radecB;
  // sorted index arrays (source index, halo bit included)
  const uint32_t* valsA;
  const uint32_t* valsB;
  // A read in place (recA64 / recA32 unused): entry p's position is the
  // keygen's (ra, dec) record of source valsA[p] (srcradA), from which the
  // filter computes the unit vector or cell record
  int a_in_place;
  const uint32_t* keysA;
  const uint32_t* keysB;
  Geom geom;
  double H_lo, H_hi;            // haversine: certain in / candidate (FP64 band)
  // A entries flagged as halo copies are skipped (partition reuse)
  int skip_halo_a;
  // self-match: A and B are one catalogue; keep pairs with a < b only
  int self_only;
  // eq. (4) per-source error radii (else nullptr): the filter ran at the
  // largest radius; each candidate is decided at k sqrt(ea^2 + eb^2)
  const double* a_err;
  const double* b_err;
  double k_sigma;
  // paper-scheme emulation (HEALPix order >= 0): keys are pixels; a pair is
  // kept in the smallest pixel its two records share
  int hp_order;
  double hp_R;
};

// Error radii of one call (nullptr a_err: a single radius).
struct Radii {
  const double* a_err;
  const double* b_err;
  double k;
};

// zero the region counters / pack the regions into the caller's buffer
// (n_pairs, n_cand and region_max of *o.cnt are set by the packing)
void launch_regions_reset(const OutArgs& o, hipStream_t s);
void launch_compact(const OutArgs& o, hipStream_t s);
// the filter writes candidates into the candidate regions; the
// certification kernel decides them and writes pairs and the band list
void launch_filter(const MatchArgs& a, const OutArgs& o, bool fp32, int items_per_wave, hipStream_t s);
void launch_cand(const MatchArgs& a, const OutArgs& o, bool fp32, hipStream_t s);
// Re-decide the band list from the original coordinates: FP64 haversine,
// then double-double inside the FP64 band.
void launch_certify(const double* a_ra, const double* a_dec, const double* b_ra,
                    const double* b_dec, double r_arcsec, double H_lo, double H_hi,
                    const Radii& rad, const OutArgs& o, hipStream_t s);
// codes (order-preserving) of the largest error of each side; err bit 8 on a
// negative or non-finite error
void launch_err_max(const double* err, uint32_t n, unsigned long long* out_code, Counters* cnt,
                    hipStream_t s);

// paper-scheme emulation: up to five (pixel, index) entries per record,
// appended after the counter *count (device)
void launch_hp_keygen(const double* ra, const double* dec, uint32_t n, int order, double R, uint32_t err_bit,
                      uint32_t* keys, uint32_t* vals, unsigned long long* count, Counters* cnt, hipStream_t s);
void launch_radec_gather(const uint32_t* vals, const DevCount& n, const double* ra, const double* dec,
                         double2* radec, hipStream_t s);
// per group of 16 A entries: B ranges of equal keys
void launch_equal_ranges(const uint32_t* keysA, const DevCount& na, const uint32_t* lb, const uint32_t* keysB,
                         const DevCount& nb, GroupRanges* out, hipStream_t s);

// ---- stream.hip ------------------------------------------------------------
// pairs[i].a += a_off for i < n
void launch_offset_pairs(uint2* pairs, uint32_t n, uint32_t a_off, hipStream_t s);

// ---- batch.hip -------------------------------------------------------------
struct BatchJob {          // one job as given by the caller, plus host-derived fields
  int64_t a_off, na, b_off, nb;
  double r_arcsec;
  double H_lo, H_hi;       // FP64 haversine band of the job's radius
  uint32_t a_entry, b_entry;  // first packed entry of the job in the A / B key arrays
  uint32_t zoff, zcap;     // the job's slice of the per-(job, zone) tables; zone budget
};
constexpr int BATCH_TILE = 1024;  // default sources per tile: 256 threads, four each
// tile sizes the batched kernels are built for (256 threads, 1, 2, 4 or 8
// sources each)
inline bool batch_tile_ok(int t) { return t == 256 || t == 512 || t == 1024 || t == 2048; }
struct BatchTile {         // <= tile consecutive sources of one job and one side
  uint32_t job, entry, src, count;
};
struct JobGeom {           // the job's local frame (computed on the device)
  double d0, h_deg, inv_h, ra0, ra_span, bin_scale, r_deg, rpad_deg;
  double c_r, t_lo64, t_hi64, H_lo, H_hi;
  double cx, cy, cz;       // FP32 frame centre (snapped)
  float thr32;
  int32_t nz, rb, full_ra;
  uint32_t nbins, zoff;
};
struct BatchMatchArgs {
  const GroupRanges* ranges;
  const uint32_t* order;   // LPT order of the groups
  unsigned int* queue;     // work-queue head
  DevCount na;
  const uint32_t* keysA;
  const uint32_t* keysB;
  const Rec64* recA64;
  const Rec64* recB64;
  const Rec32* recA32;
  const Rec32* recB32;
  const double2* radecA;
  const double2* radecB;
  const JobGeom* geo;
  int32_t lb_bits;
  unsigned long long* job_count;
};

void launch_job_bounds_init(unsigned long long* bounds, int32_t njobs, hipStream_t s);
void launch_job_bounds(const BatchTile* tiles, uint32_t ntiles, int tile, const BatchJob* jobs,
                       const double* a_ra, const double* b_ra, const double* ra, const double* dec, bool side_b,
                       unsigned long long* bounds, Counters* cnt, hipStream_t s);
void launch_job_frames(const BatchJob* jobs, int32_t njobs, const double* a_ra, const double* b_ra,
                       const unsigned long long* bounds, int32_t lb_bits, double h_factor, JobGeom* geo,
                       hipStream_t s);
void launch_batch_keygen(const BatchTile* tiles, uint32_t ntiles, int tile, const JobGeom* geo, const double* ra,
                         const double* dec, int32_t lb_bits, bool halo, uint32_t n_total, uint32_t* keys,
                         uint32_t* vals, Counters* cnt, hipStream_t s);
void launch_batch_layout32(const uint32_t* keys, const uint32_t* vals, const DevCount& n, const double* ra,
                           const double* dec, const JobGeom* geo, int32_t lb_bits, Rec32* rec,
                           double2* radec, hipStream_t s);
void launch_batch_zone_tables(const JobGeom* geo, int32_t njobs, const BatchJob* jobs, uint32_t ztotal,
                              int32_t lb_bits, const uint32_t* keysB, const DevCount& nb, int32_t* zmarg,
                              uint32_t* zstart, hipStream_t s);
void launch_batch_ranges(const uint32_t* keysA, const DevCount& na, const uint32_t* lb, const uint32_t* keysB,
                         const JobGeom* geo, int32_t lb_bits, const int32_t* zmarg, const uint32_t* zstart,
                         GroupRanges* out, uint32_t* cost_key, uint32_t* cost_val, hipStream_t s);
void launch_batch_match(const BatchMatchArgs& a, const OutArgs& o, bool fp32, uint32_t nblocks,
                        hipStream_t s);
void launch_batch_certify(const double* a_ra, const double* a_dec, const double* b_ra, const double* b_dec,
                          const BatchJob* jobs, const OutArgs& o, unsigned long long* job_count,
                          hipStream_t s);
void launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t s);

}  // namespace hlc
