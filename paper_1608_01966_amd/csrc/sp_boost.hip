// Boosting and duty cycles: Algorithm 1 multiplies each column's gated
// overlap by its boost (Section 3.2.2 computes it in the kernel); the boost
// and the permanence raise follow the whitepaper's spatial pooler phase 3.
// Exact fixed point: boosts in 1/256, duty cycles in 1/65536, updated after
// each learning frame as d <- floor((d (P - 1) + 65536 e) / P) with
// P = 2^period_log2; the minimum duty cycle is a fraction (in 1/65536) of the
// largest active duty cycle; below it the boost rises linearly to
// max_boost_q8 at duty 0; a column whose overlap duty cycle is below it has
// every permanence raised by bump_q8 / 256, clipped at 1.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kBoostThreads = 1024;
constexpr uint32_t kBoostMaxColumns = 65536;  // the library's column limit

// One workgroup: duty cycles, minimum, boosts and raise flags of one frame.
// ov: the frame's boosted overlaps (positive iff the gated overlap is);
// winners: the frame's winners (-1 padded).
__global__ __launch_bounds__(kBoostThreads) void k_boost_update(
    const int32_t* __restrict__ ov, const int32_t* __restrict__ winners, Shape sh,
    BoostParams b, uint32_t* __restrict__ adc, uint32_t* __restrict__ odc,
    uint32_t* __restrict__ boost, uint8_t* __restrict__ raise) {
  __shared__ uint32_t won[kBoostMaxColumns / 32];
  __shared__ uint32_t red[kBoostThreads / kWave];
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const uint32_t nwords = (sh.C + 31) / 32;
  for (uint32_t i = tid; i < nwords; i += kBoostThreads) won[i] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < sh.k; i += kBoostThreads) {
    const int32_t c = winners[i];
    if (c >= 0 && (uint32_t)c < sh.C) atomicOr(&won[c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  const uint64_t P = 1ull << b.period_log2;
  uint32_t mx = 0;
  for (uint32_t c = tid; c < sh.C; c += kBoostThreads) {
    const uint32_t a = (won[c >> 5] >> (c & 31)) & 1u;
    const uint32_t na = (uint32_t)(((uint64_t)adc[c] * (P - 1) + (a ? 65536u : 0u)) >> b.period_log2);
    const uint32_t no = (uint32_t)(((uint64_t)odc[c] * (P - 1) + (ov[c] > 0 ? 65536u : 0u)) >>
                                   b.period_log2);
    adc[c] = na;
    odc[c] = no;
    mx = max(mx, na);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, off));
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  mx = 0;
  for (uint32_t i = 0; i < kBoostThreads / kWave; ++i) mx = max(mx, red[i]);
  const uint32_t mn = (uint32_t)(((uint64_t)mx * b.min_pct_q16) >> 16);
  for (uint32_t c = tid; c < sh.C; c += kBoostThreads) {
    const uint32_t a = adc[c];
    boost[c] = (mn == 0 || a >= mn)
                   ? 256u
                   : 256u + (uint32_t)(((uint64_t)(b.max_boost_q8 - 256u) * (mn - a)) / mn);
    raise[c] = odc[c] < mn ? 1 : 0;
  }
}

// One wave per column: the permanence raise of flagged columns.
__global__ __launch_bounds__(256) void k_boost_raise(float* __restrict__ perm,
                                                     const uint8_t* __restrict__ raise,
                                                     Shape sh, uint32_t bump_q8) {
  const uint32_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  if (c >= sh.C || !raise[c]) return;
  float* cp = perm + (size_t)c * sh.S;
  for (uint32_t s = lane; s < sh.S; s += kWave)
    cp[s] = q_to_perm(min(perm_to_q(cp[s]) + bump_q8, 256u));
}

__global__ __launch_bounds__(256) void k_boost_init(uint32_t* __restrict__ adc,
                                                    uint32_t* __restrict__ odc,
                                                    uint32_t* __restrict__ boost, uint32_t C) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  adc[c] = 0;
  odc[c] = 0;
  boost[c] = 256;
}

}  // namespace

hipError_t launch_boost_update(const int32_t* ov, const int32_t* winners, const Shape& sh,
                               const BoostParams& b, uint32_t* adc, uint32_t* odc,
                               uint32_t* boost, uint8_t* raise, float* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_boost_update, dim3(1), dim3(kBoostThreads), 0, s, ov, winners, sh, b, adc,
                     odc, boost, raise);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.bump_q8 == 0) return e;
  hipLaunchKernelGGL(k_boost_raise, dim3((sh.C + 3) / 4), dim3(256), 0, s, perm, raise, sh,
                     b.bump_q8);
  return hipGetLastError();
}

hipError_t launch_boost_init(uint32_t* adc, uint32_t* odc, uint32_t* boost, uint32_t C,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_boost_init, dim3((C + 255) / 256), dim3(256), 0, s, adc, odc, boost, C);
  return hipGetLastError();
}

}  // namespace htmsp
