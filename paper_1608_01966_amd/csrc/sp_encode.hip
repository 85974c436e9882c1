// Adaptive video encoder (Section 3.1.2): a colour frame, optionally reduced
// in size, turned to grayscale and binarised with an adaptive threshold whose
// value at each pixel is a Gaussian-weighted sum of its neighbourhood, into
// the spatial pooler's packed input.
//
// Exact integer arithmetic throughout (so the output is bit-for-bit
// defined): block means rounded half up, BT.601 luma in 14-bit fixed point,
// the binomial window C(b-1, i) as the Gaussian (total weight 4^(b-1)),
// edge pixels repeated outside the image, mean rounded half up, on iff
// gray > mean - offset; pixel p = y w + x at bit p & 31 of word p >> 5.
//
// One workgroup per (frame, tile): a tile is a 64-pixel-aligned run of about
// kTileRows output rows in row-major order.  The workgroup builds the gray
// rows the tile needs (plus r = b/2 halo rows) in LDS straight from the RGB
// frame, the vertical window sums of the tile's rows next, and finally the
// horizontal sums, the threshold and the packing by 64-lane ballots.  Tiles
// of one frame get block ids equal modulo 8 (one XCD), so the halo rows two
// tiles share are read from device memory once.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kEncThreads = 256;

__device__ __forceinline__ uint32_t clampu(int v, uint32_t n) {
  return (uint32_t)min(max(v, 0), (int)n - 1);
}

__global__ __launch_bounds__(kEncThreads) void k_encode(const uint8_t* __restrict__ rgb,
                                                        uint32_t F, EncShape e,
                                                        uint32_t* __restrict__ out) {
  extern __shared__ uint32_t lds[];
  const uint32_t per = 8 * e.tiles;
  const uint32_t f = (blockIdx.x / per) * 8 + blockIdx.x % 8;
  const uint32_t tile = (blockIdx.x % per) / 8;
  if (f >= F) return;  // whole workgroup
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const uint32_t w = e.w, h = e.h, r = e.block / 2;
  const uint32_t p0 = tile * e.tile_px;
  const uint32_t p1 = min(p0 + e.tile_px, w * h);
  const uint32_t ya = p0 / w, yb = (p1 - 1) / w;        // output rows of the tile
  const uint32_t ga = ya >= r ? ya - r : 0u;            // gray rows held
  const uint32_t gb = min(yb + r, h - 1);
  const uint32_t grows = gb - ga + 1, vrows = yb - ya + 1;
  uint8_t* G = reinterpret_cast<uint8_t*>(lds);                          // [grows][w]
  uint32_t* V = lds + (e.gray_bytes + 3) / 4;                            // [vrows][w]

  // binomial weights (row b - 1 of Pascal's triangle)
  uint32_t wt[11];
  wt[0] = 1;
#pragma unroll
  for (uint32_t i = 1; i < 11; ++i) wt[i] = i < e.block ? wt[i - 1] * (e.block - i) / i : 0u;

  // Gray rows [ga, gb]: block means of the RGB input, then luma.
  const uint8_t* src = rgb + (size_t)f * e.W * e.H * 3;
  const uint32_t fa = e.factor, area = fa * fa;
  for (uint32_t i = tid; i < grows * w; i += kEncThreads) {
    const uint32_t gy = ga + i / w, gx = i % w;
    uint32_t R = 0, Gc = 0, B = 0;
    for (uint32_t dy = 0; dy < fa; ++dy) {
      const uint8_t* row = src + 3 * ((size_t)(gy * fa + dy) * e.W + gx * fa);
      for (uint32_t dx = 0; dx < fa; ++dx) {
        R += row[3 * dx];
        Gc += row[3 * dx + 1];
        B += row[3 * dx + 2];
      }
    }
    R = (R + area / 2) / area;
    Gc = (Gc + area / 2) / area;
    B = (B + area / 2) / area;
    G[i] = (uint8_t)((4899u * R + 9617u * Gc + 1868u * B + 8192u) >> 14);
  }
  __syncthreads();

  // Vertical window sums of the tile's rows.
  for (uint32_t i = tid; i < vrows * w; i += kEncThreads) {
    const uint32_t y = ya + i / w, x = i % w;
    uint32_t s = 0;
    for (uint32_t k = 0; k < e.block; ++k)
      s += wt[k] * G[(clampu((int)(y + k) - (int)r, h) - ga) * w + x];
    V[i] = s;
  }
  __syncthreads();

  // Horizontal sums, threshold, and packing: 64 consecutive pixels per wave
  // per round, two output words from one ballot.
  const uint32_t shift = 2 * (e.block - 1);
  const uint32_t half = 1u << (shift - 1);
  for (uint32_t q0 = p0 + kWave * wave; q0 < p1; q0 += kEncThreads) {
    const uint32_t p = q0 + lane;
    bool on = false;
    if (p < p1) {
      const uint32_t y = p / w, x = p % w;
      const uint32_t* vr = V + (y - ya) * w;
      uint32_t s = 0;
      for (uint32_t k = 0; k < e.block; ++k)
        s += wt[k] * vr[clampu((int)(x + k) - (int)r, w)];
      const int mean = (int)((s + half) >> shift);
      on = (int)G[(y - ga) * w + x] > mean - e.offset;
    }
    const uint64_t bits = __ballot(on);
    const uint32_t word = q0 / 32;  // q0 is a multiple of 64
    uint32_t* dst = out + (size_t)f * e.words;
    if (lane == 0) dst[word] = (uint32_t)bits;
    if (lane == 1 && q0 + 32 < p1) dst[word + 1] = (uint32_t)(bits >> 32);
  }
}

}  // namespace

hipError_t launch_encode(const uint8_t* rgb, uint32_t F, const EncShape& e, uint32_t* out,
                         hipStream_t s) {
  if (F == 0) return hipSuccess;
  if (e.lds_bytes > 65536) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_encode),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)e.lds_bytes);
    if (err != hipSuccess) return err;
  }
  const uint32_t groups = (F + 7) / 8 * 8;
  hipLaunchKernelGGL(k_encode, dim3(groups * e.tiles), dim3(kEncThreads), e.lds_bytes, s, rgb,
                     F, e, out);
  return hipGetLastError();
}

}  // namespace htmsp
