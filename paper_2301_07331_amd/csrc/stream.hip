// stream.hip -- kernels of the streaming form: catalogues arrive from pinned
// host memory in slabs (section 4.3.1: copies on their own stream overlap the
// device work; section 4.3.2: page-locked host memory), are bucketed on the
// device into declination chunks (a second-level partition bounded by device
// memory, as section 4.2 bounds its calculation blocks), and each chunk's
// pairs pass through a bounded device ring back to the host.
//
// A source belongs to the chunk holding its Dec; a B source also goes to every
// chunk whose Dec range padded by r reaches it, so each pair is found exactly
// once, in the chunk of its A source.
#include <hip/hip_runtime.h>

#include "hlc_kernels.hpp"

namespace hlc {

namespace {

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Fine Dec histogram bin of a declination (NBINS bins over [-90, 90]).
__device__ inline int32_t dec_bin(double dec, int32_t nbins) {
  double t = floor((dec + 90.0) * ((double)nbins / 180.0));
  if (!(t >= 0.0)) return 0;
  if (t > (double)(nbins - 1)) return nbins - 1;
  return (int32_t)t;
}

// Sources per block; counts are gathered in LDS and added to the global
// bins once per block (a catalogue confined to a few degrees of Dec would
// otherwise send every source's atomic to the same few addresses).
constexpr int SB_ITEMS = 16;
constexpr uint32_t SB_TILE = 256u * SB_ITEMS;
constexpr int32_t LDS_BINS = 8192;   // k_dec_hist: 32 KB
constexpr int32_t LDS_CHUNKS = 4096;  // k_chunk_scatter: at most 48 KB

__global__ __launch_bounds__(256) void k_dec_hist(const double* __restrict__ ra,
                                                  const double* __restrict__ dec, uint32_t n,
                                                  int32_t nbins, uint32_t* __restrict__ hist,
                                                  uint32_t err_bit, Counters* cnt) {
  __shared__ uint32_t h[LDS_BINS];
  for (int32_t k = threadIdx.x; k < nbins; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  const uint32_t base = blockIdx.x * SB_TILE;
  bool bad = false;
  for (int j = 0; j < SB_ITEMS; ++j) {
    const uint32_t i = base + (uint32_t)j * 256u + threadIdx.x;
    if (i >= n) break;
    const double a = ra[i], d = dec[i];
    if (!valid_pos(a, d)) {
      bad = true;
      continue;
    }
    atomicAdd(&h[dec_bin(d, nbins)], 1u);
  }
  if (bad) atomicOr(&cnt->err, err_bit);
  __syncthreads();
  for (int32_t k = threadIdx.x; k < nbins; k += blockDim.x)
    if (h[k]) atomicAdd(&hist[k], h[k]);
}

// Scatter sources into chunk-ordered arrays. chunk_of_bin maps a fine Dec bin
// to its chunk; chunk edges in degrees are edges[c], edges[c+1]. With
// `halo_deg` > 0 a source is also written to every other chunk whose range
// padded by halo_deg contains it.
// Per block: the block's entries per chunk are counted in LDS, each chunk's
// cursor is advanced once, and entries take consecutive slots of their
// chunk's run (in no particular order inside the block).
__device__ inline void chunk_span(double d, int32_t nbins, const int32_t* chunk_of_bin, const double* edges,
                                  int32_t nchunks, double halo_deg, int32_t& c0, int32_t& c1) {
  const int32_t c = chunk_of_bin[dec_bin(d, nbins)];
  c0 = c;
  c1 = c;
  if (halo_deg > 0.0) {
    while (c0 > 0 && d - halo_deg <= edges[c0]) --c0;
    while (c1 < nchunks - 1 && d + halo_deg >= edges[c1 + 1]) ++c1;
  }
}

__global__ __launch_bounds__(256) void k_chunk_scatter(
    const double* __restrict__ ra, const double* __restrict__ dec, uint32_t n, uint32_t base_index,
    int32_t nbins, const int32_t* __restrict__ chunk_of_bin, const double* __restrict__ edges,
    int32_t nchunks, double halo_deg, unsigned long long* __restrict__ cursor,
    double* __restrict__ out_ra, double* __restrict__ out_dec, uint32_t* __restrict__ out_idx) {
  // dynamic LDS: nchunks bases (u64) then nchunks counts (u32)
  extern __shared__ unsigned long long s_dyn[];
  unsigned long long* s_base = s_dyn;
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_dyn + nchunks);
  for (int32_t k = threadIdx.x; k < nchunks; k += blockDim.x) s_cnt[k] = 0u;
  __syncthreads();
  const uint32_t base = blockIdx.x * SB_TILE;
  for (int j = 0; j < SB_ITEMS; ++j) {
    const uint32_t i = base + (uint32_t)j * 256u + threadIdx.x;
    if (i >= n) break;
    const double a = ra[i], d = dec[i];
    if (!valid_pos(a, d)) continue;
    int32_t c0, c1;
    chunk_span(d, nbins, chunk_of_bin, edges, nchunks, halo_deg, c0, c1);
    for (int32_t k = c0; k <= c1; ++k) atomicAdd(&s_cnt[k], 1u);
  }
  __syncthreads();
  for (int32_t k = threadIdx.x; k < nchunks; k += blockDim.x) {
    s_base[k] = s_cnt[k] ? atomicAdd(&cursor[k], (unsigned long long)s_cnt[k]) : 0ull;
    s_cnt[k] = 0u;
  }
  __syncthreads();
  if (out_ra == nullptr) return;  // counting pass
  for (int j = 0; j < SB_ITEMS; ++j) {
    const uint32_t i = base + (uint32_t)j * 256u + threadIdx.x;
    if (i >= n) break;
    const double a = ra[i], d = dec[i];
    if (!valid_pos(a, d)) continue;
    int32_t c0, c1;
    chunk_span(d, nbins, chunk_of_bin, edges, nchunks, halo_deg, c0, c1);
    for (int32_t k = c0; k <= c1; ++k) {
      const unsigned long long pos = s_base[k] + atomicAdd(&s_cnt[k], 1u);
      out_ra[pos] = a;
      out_dec[pos] = d;
      out_idx[pos] = base_index + i;
    }
  }
}

// The same with one atomic per entry (more chunks than the LDS holds).
__global__ __launch_bounds__(256) void k_chunk_scatter_atomic(
    const double* __restrict__ ra, const double* __restrict__ dec, uint32_t n, uint32_t base_index,
    int32_t nbins, const int32_t* __restrict__ chunk_of_bin, const double* __restrict__ edges,
    int32_t nchunks, double halo_deg, unsigned long long* __restrict__ cursor,
    double* __restrict__ out_ra, double* __restrict__ out_dec, uint32_t* __restrict__ out_idx) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = ra[i], d = dec[i];
  if (!valid_pos(a, d)) return;
  int32_t c0, c1;
  chunk_span(d, nbins, chunk_of_bin, edges, nchunks, halo_deg, c0, c1);
  for (int32_t k = c0; k <= c1; ++k) {
    const unsigned long long pos = atomicAdd(&cursor[k], 1ull);
    if (out_ra == nullptr) continue;  // counting pass
    out_ra[pos] = a;
    out_dec[pos] = d;
    out_idx[pos] = base_index + i;
  }
}

// Chunk-local pair indices -> original indices.
__global__ __launch_bounds__(256) void k_remap_pairs(uint2* __restrict__ pairs, uint32_t n,
                                                     const uint32_t* __restrict__ a_idx,
                                                     const uint32_t* __restrict__ b_idx) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint2 p = pairs[i];
  pairs[i] = make_uint2(a_idx[p.x], b_idx[p.y]);
}

}  // namespace

void launch_dec_hist(const double* ra, const double* dec, uint32_t n, int32_t nbins, uint32_t* hist,
                     uint32_t err_bit, Counters* cnt, hipStream_t s) {
  if (n == 0 || nbins > LDS_BINS) return;
  k_dec_hist<<<cdiv(n, SB_TILE), 256, 0, s>>>(ra, dec, n, nbins, hist, err_bit, cnt);
}

void launch_chunk_scatter(const double* ra, const double* dec, uint32_t n, uint32_t base_index,
                          int32_t nbins, const int32_t* chunk_of_bin, const double* edges,
                          int32_t nchunks, double halo_deg, unsigned long long* cursor,
                          double* out_ra, double* out_dec, uint32_t* out_idx, hipStream_t s) {
  if (n == 0) return;
  if (nchunks <= LDS_CHUNKS) {
    const size_t lds = (size_t)nchunks * (sizeof(unsigned long long) + sizeof(uint32_t));
    k_chunk_scatter<<<cdiv(n, SB_TILE), 256, lds, s>>>(ra, dec, n, base_index, nbins, chunk_of_bin, edges,
                                                        nchunks, halo_deg, cursor, out_ra, out_dec, out_idx);
  } else {
    k_chunk_scatter_atomic<<<cdiv(n, 256), 256, 0, s>>>(ra, dec, n, base_index, nbins, chunk_of_bin, edges,
                                                         nchunks, halo_deg, cursor, out_ra, out_dec, out_idx);
  }
}

void launch_remap_pairs(uint2* pairs, uint32_t n, const uint32_t* a_idx, const uint32_t* b_idx,
                        hipStream_t s) {
  if (n == 0) return;
  k_remap_pairs<<<cdiv(n, 256), 256, 0, s>>>(pairs, n, a_idx, b_idx);
}

}  // namespace hlc
