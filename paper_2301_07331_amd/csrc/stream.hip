// stream.hip -- kernels of the streaming form. The catalogues arrive from
// pinned host memory (section 4.3.2: page-locked host memory): B once, A in
// slabs of consecutive sources whose copies, on their own stream, overlap the
// cross-match of the previous slab (section 4.3.1). Each slab's pairs pass
// through a bounded device ring back to the host; their A indices are local
// to the slab until the kernel below makes them global.
#include <hip/hip_runtime.h>

#include "hlc_kernels.hpp"

namespace hlc {

namespace {

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// pairs[i].a += a_off (A indices of a slab become indices into the whole A)
__global__ __launch_bounds__(256) void k_offset_pairs(uint2* __restrict__ pairs, uint32_t n, uint32_t a_off) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pairs[i].x += a_off;
}

}  // namespace

void launch_offset_pairs(uint2* pairs, uint32_t n, uint32_t a_off, hipStream_t s) {
  if (n == 0 || a_off == 0) return;
  k_offset_pairs<<<cdiv(n, 256), 256, 0, s>>>(pairs, n, a_off);
}

}  // namespace hlc
