// RPA_POISON debugging mode: new device allocations are filled with 0xFF bytes, so that a
// kernel that reads a workspace element before writing it produces NaN instead of
// whatever the memory held (tests compare poisoned and ordinary runs bit for bit).
#include <algorithm>

#include "common.hpp"

namespace rpa {

namespace {
__global__ void poison_kernel(uint4 *p16, int64_t n16, unsigned char *tail, int64_t ntail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p16[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
  if (blockIdx.x == 0 && (int64_t)threadIdx.x < ntail) tail[threadIdx.x] = 0xFF;
}
}  // namespace

hipError_t launch_poison_fill(hipStream_t s, void *p, int64_t bytes) {
  if (!p || bytes <= 0) return hipSuccess;
  // hipMalloc returns 256-byte aligned memory; the last bytes % 16 are written one by one
  const int64_t n16 = bytes / 16, ntail = bytes % 16;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n16 + 255) / 256, 4096));
  hipLaunchKernelGGL(poison_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint4 *)p, n16,
                     (unsigned char *)p + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace rpa
