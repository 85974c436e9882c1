// Per-stream SDR histograms (Section 2: the pooler output of every frame of a
// video is accumulated into a histogram that serves as the video's feature
// vector).  Adds 1 to hist[c] for every winner entry c >= 0 of a call's
// [F][k] winners.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

__global__ __launch_bounds__(256) void k_hist_add(const int32_t* __restrict__ winners, size_t n,
                                                  uint32_t C, uint32_t* __restrict__ hist) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int32_t c = winners[i];
    if (c >= 0 && (uint32_t)c < C) atomicAdd(&hist[c], 1u);
  }
}

}  // namespace

hipError_t launch_hist_add(const int32_t* winners, size_t n, uint32_t C, uint32_t* hist,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_hist_add, dim3((uint32_t)blocks), dim3(256), 0, s, winners, n, C, hist);
  return hipGetLastError();
}

}  // namespace htmsp
