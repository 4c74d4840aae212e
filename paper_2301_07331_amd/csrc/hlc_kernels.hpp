// hlc_kernels.hpp -- host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hlc_device.hpp"

namespace hlc {

// ---- partition.hip ---------------------------------------------------------
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void launch_zero_counters(Counters* c, hipStream_t s);
// keys/vals for A (one entry per source, or one per source plus Dec-halo
// copies appended after n when `halo` is set).
void launch_keygen(const double* ra, const double* dec, uint32_t n, const Geom& g, bool halo,
                   uint32_t err_bit, uint32_t* keys, uint32_t* vals, Counters* cnt, hipStream_t s);

struct SortScratch {
  uint32_t* keys_alt;
  uint32_t* vals_alt;
  uint32_t* counts;     // 256 * ntiles
  uint32_t* block_sums; // scan partials
};
size_t sort_counts_len(uint32_t n);
size_t sort_block_sums_len(uint32_t n);
// LSD radix sort of (keys, vals), ascending, stable, on key bits [0, key_bits).
// The result ends in (keys, vals).
void radix_sort(uint32_t* keys, uint32_t* vals, uint32_t n, int key_bits, const SortScratch& sc,
                hipStream_t s);

void launch_zone_tables(const Geom& g, int32_t* zmarg, double2* zone_cs, double2* super_cs,
                        hipStream_t s);
void launch_zone_starts(const uint32_t* keys, uint32_t n, const Geom& g, uint32_t* zstart,
                        hipStream_t s);
void launch_layout64(const uint32_t* vals, uint32_t n, const double* ra, const double* dec,
                     Rec64* rec, hipStream_t s);
void launch_layout32(const uint32_t* keys, const uint32_t* vals, uint32_t n, const double* ra,
                     const double* dec, const Geom& g, const double2* zone_cs,
                     const double2* super_cs, Rec32* rec, double2* radec, hipStream_t s);
void launch_merge_lb(const uint32_t* keysA, uint32_t na, const uint32_t* keysB, uint32_t nb,
                     uint32_t* lb, hipStream_t s);
void launch_ranges(const uint32_t* keysA, uint32_t na, const uint32_t* lb, const uint32_t* keysB,
                   uint32_t nb, const uint32_t* zstartB, const int32_t* zmarg, const Geom& g,
                   double c_r, GroupRanges* out, hipStream_t s);

// ---- match.hip -------------------------------------------------------------
struct OutArgs {
  uint2* pairs;                 // caller buffer (a, b)
  double* sep;                  // caller buffer or nullptr
  unsigned long long cap;       // capacity in pairs
  uint2* band;                  // band list (original indices, B halo bit cleared)
  unsigned long long band_cap;
  Counters* cnt;
};

struct MatchArgs {
  const GroupRanges* ranges;
  uint32_t na, nb;
  // FP64 form
  const Rec64* recA64;
  const Rec64* recB64;
  double t_lo64, t_hi64;        // chord^2: certain in / candidate
  // FP32 form
  const Rec32* recA32;
  const Rec32* recB32;
  const double2* radecA;
  const double2* radecB;
  const uint32_t* keysA;
  const uint32_t* keysB;
  const double2* zone_cs;
  const double2* super_cs;
  Geom geom;
  double H_lo, H_hi;            // haversine: certain in / candidate (FP64 band)
  // A entries flagged as halo copies are skipped (partition reuse)
  int skip_halo_a;
  // self-match: A and B are one catalogue; keep pairs with a < b only
  int self_only;
};

void launch_match64(const MatchArgs& a, const OutArgs& o, hipStream_t s);
void launch_match32(const MatchArgs& a, const OutArgs& o, hipStream_t s);
// Re-decide the band list from the original coordinates: FP64 haversine,
// then double-double inside the FP64 band.
void launch_certify(const double* a_ra, const double* a_dec, const double* b_ra,
                    const double* b_dec, double r_arcsec, double H_lo, double H_hi,
                    const OutArgs& o, hipStream_t s);

}  // namespace hlc
