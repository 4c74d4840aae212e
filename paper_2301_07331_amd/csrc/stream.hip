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

__global__ __launch_bounds__(256) void k_dec_hist(const double* __restrict__ ra,
                                                  const double* __restrict__ dec, uint32_t n,
                                                  int32_t nbins, uint32_t* __restrict__ hist,
                                                  uint32_t err_bit, Counters* cnt) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = ra[i], d = dec[i];
  if (!valid_pos(a, d)) {
    atomicOr(&cnt->err, err_bit);
    return;
  }
  atomicAdd(&hist[dec_bin(d, nbins)], 1u);
}

// Scatter sources into chunk-ordered arrays. chunk_of_bin maps a fine Dec bin
// to its chunk; chunk edges in degrees are edges[c], edges[c+1]. With
// `halo_deg` > 0 a source is also written to every other chunk whose range
// padded by halo_deg contains it.
__global__ __launch_bounds__(256) void k_chunk_scatter(
    const double* __restrict__ ra, const double* __restrict__ dec, uint32_t n, uint32_t base_index,
    int32_t nbins, const int32_t* __restrict__ chunk_of_bin, const double* __restrict__ edges,
    int32_t nchunks, double halo_deg, unsigned long long* __restrict__ cursor,
    double* __restrict__ out_ra, double* __restrict__ out_dec, uint32_t* __restrict__ out_idx) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = ra[i], d = dec[i];
  if (!valid_pos(a, d)) return;
  int32_t c = chunk_of_bin[dec_bin(d, nbins)];
  int32_t c0 = c, c1 = c;
  if (halo_deg > 0.0) {
    while (c0 > 0 && d - halo_deg <= edges[c0]) --c0;
    while (c1 < nchunks - 1 && d + halo_deg >= edges[c1 + 1]) ++c1;
  }
  for (int32_t k = c0; k <= c1; ++k) {
    unsigned long long pos = atomicAdd(&cursor[k], 1ull);
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
  if (n == 0) return;
  k_dec_hist<<<cdiv(n, 256), 256, 0, s>>>(ra, dec, n, nbins, hist, err_bit, cnt);
}

void launch_chunk_scatter(const double* ra, const double* dec, uint32_t n, uint32_t base_index,
                          int32_t nbins, const int32_t* chunk_of_bin, const double* edges,
                          int32_t nchunks, double halo_deg, unsigned long long* cursor,
                          double* out_ra, double* out_dec, uint32_t* out_idx, hipStream_t s) {
  if (n == 0) return;
  k_chunk_scatter<<<cdiv(n, 256), 256, 0, s>>>(ra, dec, n, base_index, nbins, chunk_of_bin, edges,
                                                nchunks, halo_deg, cursor, out_ra, out_dec, out_idx);
}

void launch_remap_pairs(uint2* pairs, uint32_t n, const uint32_t* a_idx, const uint32_t* b_idx,
                        hipStream_t s) {
  if (n == 0) return;
  k_remap_pairs<<<cdiv(n, 256), 256, 0, s>>>(pairs, n, a_idx, b_idx);
}

}  // namespace hlc
