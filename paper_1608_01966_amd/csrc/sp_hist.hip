// Per-stream SDR histograms (Section 2: the pooler output of every frame of a
// video is accumulated into a histogram that serves as the video's feature
// vector).  Adds 1 to hist[c] for every winner entry c >= 0 of a call's
// [F][k] winners, or, for the local-inhibition step whose output is an
// active mask, for every frame in which column c is active.
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

// Column c of every frame of an [F][C] 0/1 mask: thread per column, frames
// summed in a register, one add per column.
__global__ __launch_bounds__(256) void k_hist_add_active(const uint8_t* __restrict__ active,
                                                         uint32_t F, uint32_t C,
                                                         uint32_t* __restrict__ hist) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  uint32_t n = 0;
  for (uint32_t t = 0; t < F; ++t) n += active[(size_t)t * C + c] != 0;
  if (n) hist[c] += n;
}

}  // namespace

hipError_t launch_hist_add_active(const uint8_t* active, uint32_t F, uint32_t C, uint32_t* hist,
                                  hipStream_t s) {
  if (F == 0 || C == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist_add_active, dim3((C + 255) / 256), dim3(256), 0, s, active, F, C,
                     hist);
  return hipGetLastError();
}

hipError_t launch_hist_add(const int32_t* winners, size_t n, uint32_t C, uint32_t* hist,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_hist_add, dim3((uint32_t)blocks), dim3(256), 0, s, winners, n, C, hist);
  return hipGetLastError();
}

}  // namespace htmsp
