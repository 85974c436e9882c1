// Local inhibition: Algorithm 2 as printed, each column competing within a
// neighbourhood given by an inhibition radius (the form Section 3.2.2
// describes), and the learning step built on it.
//
// Columns sit on a row-major grid of grid_w columns per row.  The
// neighbourhood of c is every other column within `radius` in both grid
// coordinates (no wrap-around); with v the n-th largest neighbour overlap
// (0 when there are fewer than n neighbours), c is active iff its overlap is
// greater than max(v, 1).  Equivalently -- and that is what the kernel
// counts -- c is active iff its overlap is at least 2 and fewer than n
// neighbours have an overlap at least as large; a thread stops counting as
// soon as n are found, so most columns (low overlaps) finish early.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kLocalThreads = 256;
constexpr uint32_t kLocalLdsColumns = 16384;  // a frame's overlaps fit LDS up to this C

// Block (frame f, columns [b * 256, b * 256 + 256)).  LDS: the whole frame's
// overlaps when they fit, else reads from device memory.
template <bool LDS>
__global__ __launch_bounds__(kLocalThreads) void k_inhibit_local(
    const int32_t* __restrict__ ov, uint32_t C, uint32_t grid_w, uint32_t radius, uint32_t n,
    uint32_t col_blocks, uint8_t* __restrict__ active) {
  __shared__ int32_t s_ov[LDS ? kLocalLdsColumns : 1];
  const uint32_t f = blockIdx.x / col_blocks;
  const uint32_t c = (blockIdx.x % col_blocks) * kLocalThreads + threadIdx.x;
  const int32_t* o = ov + (size_t)f * C;
  if constexpr (LDS) {
    for (uint32_t i = threadIdx.x; i < C; i += kLocalThreads) s_ov[i] = o[i];
    __syncthreads();
  }
  if (c >= C) return;
  const int32_t* src = LDS ? s_ov : o;
  const int32_t v = src[c];
  uint8_t on = 0;
  if (v >= 2) {
    const uint32_t rows = (C + grid_w - 1) / grid_w;
    const uint32_t cx = c % grid_w, cy = c / grid_w;
    const uint32_t y0 = cy >= radius ? cy - radius : 0u;
    const uint32_t y1 = min(cy + radius, rows - 1);
    const uint32_t x0 = cx >= radius ? cx - radius : 0u;
    const uint32_t x1 = min(cx + radius, grid_w - 1);
    uint32_t k = 0;
    for (uint32_t y = y0; y <= y1 && k < n; ++y) {
      const uint32_t base = y * grid_w;
      for (uint32_t x = x0; x <= x1; ++x) {
        const uint32_t d = base + x;
        if (d >= C) break;  // the last grid row may be partly empty
        k += (d != c && src[d] >= v) ? 1u : 0u;
      }
    }
    on = k < n ? 1 : 0;
  }
  active[(size_t)f * C + c] = on;
}

// Learning on the active columns of one frame: one wave per column, idle
// for inactive ones.
__global__ __launch_bounds__(256) void k_learn_active(const uint32_t* __restrict__ idx,
                                                      float* __restrict__ perm,
                                                      const uint32_t* __restrict__ frame,
                                                      const uint8_t* __restrict__ active,
                                                      Shape sh) {
  const uint32_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  if (c >= sh.C || !active[c]) return;
  const uint32_t* ci = idx + (size_t)c * sh.S;
  float* cp = perm + (size_t)c * sh.S;
  for (uint32_t s = lane; s < sh.S; s += kWave) {
    const uint32_t i = min(ci[s], sh.N - 1);
    cp[s] = q_to_perm(learn_q(perm_to_q(cp[s]), input_bit(frame[i >> 5], i), sh));
  }
}

}  // namespace

hipError_t launch_inhibit_local(const int32_t* ov, uint32_t F, uint32_t C, uint32_t grid_w,
                                uint32_t radius, uint32_t n, uint8_t* active, hipStream_t s) {
  if (F == 0) return hipSuccess;
  const uint32_t col_blocks = (C + kLocalThreads - 1) / kLocalThreads;
  const dim3 grid(F * col_blocks);
  if (C <= kLocalLdsColumns)
    hipLaunchKernelGGL(k_inhibit_local<true>, grid, dim3(kLocalThreads), 0, s, ov, C, grid_w,
                       radius, n, col_blocks, active);
  else
    hipLaunchKernelGGL(k_inhibit_local<false>, grid, dim3(kLocalThreads), 0, s, ov, C, grid_w,
                       radius, n, col_blocks, active);
  return hipGetLastError();
}

hipError_t launch_learn_active(const uint32_t* idx, float* perm, const uint32_t* frame,
                               const uint8_t* active, const Shape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_active, dim3((sh.C + 3) / 4), dim3(256), 0, s, idx, perm, frame,
                     active, sh);
  return hipGetLastError();
}

}  // namespace htmsp
