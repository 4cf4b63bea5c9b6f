// The generator's raw output for checking it against an independent
// implementation: the four 64-bit words of Philox4x64-10 for a run of
// consecutive counters, written to a device array.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/picmcc.h"
#include "philox.h"
#include "pm_internal.h"

namespace pm {

__global__ __launch_bounds__(kBlock) void k_philox_words(uint64_t id0, uint64_t index, uint64_t tag, uint64_t aux,
                                                         uint64_t key0, uint64_t key1, int64_t n,
                                                         uint64_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const Words4 w = philox4x64_10(id0 + (uint64_t)i, index, tag, aux, key0, key1);
    out[4 * i + 0] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
  }
}

}  // namespace pm

pm_status pm_philox_words(uint64_t id0, uint64_t index, uint64_t tag, uint64_t aux, uint64_t seed,
                          uint64_t stream_key, int64_t n, uint64_t* out_dev, void* hip_stream) {
  if (n < 0 || (n > 0 && !out_dev)) return PM_EINVAL;
  if (n == 0) return PM_OK;
  const int64_t blocks = std::min<int64_t>((n + pm::kBlock - 1) / pm::kBlock, 4096);
  hipLaunchKernelGGL(pm::k_philox_words, dim3((unsigned)blocks), dim3(pm::kBlock), 0,
                     reinterpret_cast<hipStream_t>(hip_stream), id0, index, tag, aux, seed, stream_key, n, out_dev);
  return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}
