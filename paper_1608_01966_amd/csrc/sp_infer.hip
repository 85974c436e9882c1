// Batched inference: F independent frames through a spatial pooler whose
// state is frozen (learning off, Section 4.1's testing mode), overlap and
// inhibition per frame (Section 1.1, Algorithms 1 and 2, global form).
//
// With learning off every frame sees the same connected synapses, so a prep
// kernel compacts each column's connected inputs once into a slot-major list.
// The gather kernel then holds one column per thread, its list in registers,
// stages one whole frame at a time in LDS (a 960x540 frame is 64 800 B), and
// counts the connected inputs that are on with one LDS read each; the
// workgroups that share a frame run on one XCD so its L2 serves them all.
// Columns with more connected synapses than the registers hold read their
// lists from device memory instead (k_infer_gather_long).
// A second kernel resolves the global top-k of every frame, one wave per
// frame, on overlaps packed four per 64-bit word.
#include <type_traits>

#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kInferThreads = 256;

// List entry for input pixel p: its frame word in the high bits, its bit in
// the low five, so one shift gives the word and a bit-field extract (which
// reads only the low five bits of its offset) gives the bit.
__device__ __forceinline__ uint32_t list_entry(uint32_t p) { return ((p >> 5) << 7) | (p & 31u); }
__device__ __forceinline__ uint32_t entry_word(uint32_t e) { return e >> 7; }
// The word of entry e in a frame staged at `fr`: bits 5 and 6 of an entry are
// zero, so e >> 5 is already the word's byte offset (one shift, no mask).
__device__ __forceinline__ uint32_t entry_load(const uint32_t* fr, uint32_t e) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(fr) + (e >> 5));
}

// Column c's connected inputs, slot-major: list[i * C + c] for i < cnt[c];
// slots from cnt[c] to S - 1 hold `pad`, the entry of a word that is always
// zero (one past the frame).
__global__ __launch_bounds__(256) void k_infer_prep(const uint32_t* __restrict__ idx,
                                                    const float* __restrict__ perm, Shape sh,
                                                    uint32_t pad, uint32_t* __restrict__ list,
                                                    uint32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ maxcnt) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= sh.C) return;
  uint32_t n = 0;
  for (uint32_t s = 0; s < sh.S; ++s) {
    const size_t off = (size_t)c * sh.S + s;
    if (perm_to_q(perm[off]) >= sh.theta)
      list[(size_t)n++ * sh.C + c] = list_entry(min(idx[off], sh.N - 1));
  }
  cnt[c] = n;
  for (uint32_t i = n; i < sh.S; ++i) list[(size_t)i * sh.C + c] = pad;
  if (maxcnt) atomicMax(maxcnt, n);
}

// Gather overlaps.  Block b serves column block cb (kInferThreads columns)
// for frame group fg; the col_blocks blocks of one frame group get ids that
// are equal modulo 8, i.e. run on one XCD.  LDS == true stages each frame
// (W words plus the zero padding word) in LDS; otherwise words are read
// from global memory (frames too large for LDS).
template <int MAXN, bool LDS>
__global__ __launch_bounds__(kInferThreads) void k_infer_gather(
    const uint32_t* __restrict__ frames, uint32_t F, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ cnt, Shape sh, uint32_t frames_per_group, uint32_t col_blocks,
    uint32_t groups, int32_t* __restrict__ ov_out) {
  extern __shared__ uint32_t fr[];
  const uint32_t per = 8 * col_blocks;
  const uint32_t fg = (blockIdx.x / per) * 8 + blockIdx.x % 8;
  const uint32_t cb = (blockIdx.x % per) / 8;
  if (fg >= groups) return;
  const uint32_t c = cb * kInferThreads + threadIdx.x;
  const bool col_ok = c < sh.C;
  const uint32_t pad = sh.W << 7;

  uint32_t lst[MAXN];
#pragma unroll
  for (int i = 0; i < MAXN; ++i)
    lst[i] = (col_ok && (uint32_t)i < sh.S) ? list[(size_t)i * sh.C + c] : pad;
  uint32_t n = col_ok ? cnt[c] : 0u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n = max(n, (uint32_t)__shfl_xor(n, off));

  const uint32_t f0 = fg * frames_per_group;
  const uint32_t f1 = min(F, f0 + frames_per_group);
  for (uint32_t f = f0; f < f1; ++f) {
    const uint32_t* frame = frames + (size_t)f * sh.W;
    if constexpr (LDS) {
      __syncthreads();
      const uint32_t w4 = sh.W / 4;
      const uint4* src = reinterpret_cast<const uint4*>(frame);
      if ((reinterpret_cast<uintptr_t>(frame) & 15u) == 0) {
        for (uint32_t i = threadIdx.x; i < w4; i += kInferThreads)
          reinterpret_cast<uint4*>(fr)[i] = src[i];
        for (uint32_t i = 4 * w4 + threadIdx.x; i < sh.W; i += kInferThreads) fr[i] = frame[i];
      } else {
        for (uint32_t i = threadIdx.x; i < sh.W; i += kInferThreads) fr[i] = frame[i];
      }
      if (threadIdx.x == 0) fr[sh.W] = 0u;
      __syncthreads();
    }
    // Keep one register per list entry: the empty asm stops the compiler
    // from hoisting each entry's word address out of the frame loop.
#pragma unroll
    for (int i = 0; i < MAXN; ++i) asm volatile("" : "+v"(lst[i]));
    uint32_t acc = 0;
#pragma unroll
    for (int i0 = 0; i0 < MAXN; i0 += 16) {
      if ((uint32_t)i0 < n) {
#pragma unroll
        for (int i = i0; i < i0 + 16; ++i) {
          const uint32_t e = lst[i];
          const uint32_t wi = entry_word(e);
          const uint32_t word = LDS ? entry_load(fr, e) : (wi < sh.W ? frame[wi] : 0u);
          acc += __builtin_amdgcn_ubfe(word, e, 1);
        }
      }
    }
    if (col_ok) ov_out[(size_t)f * sh.C + c] = acc >= sh.m ? (int32_t)acc : 0;
  }
}

// Gather overlaps for lists longer than the register-resident kernels hold:
// the same block mapping and frame staging as k_infer_gather, but each
// thread reads its column's list entries from device memory for every frame
// (slot-major, so a wave's reads of one slot are coalesced; the lists stay
// in L2 across the frames of a group).
template <bool LDS>
__global__ __launch_bounds__(kInferThreads) void k_infer_gather_long(
    const uint32_t* __restrict__ frames, uint32_t F, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ cnt, Shape sh, uint32_t frames_per_group, uint32_t col_blocks,
    uint32_t groups, int32_t* __restrict__ ov_out) {
  extern __shared__ uint32_t fr[];
  const uint32_t per = 8 * col_blocks;
  const uint32_t fg = (blockIdx.x / per) * 8 + blockIdx.x % 8;
  const uint32_t cb = (blockIdx.x % per) / 8;
  if (fg >= groups) return;  // whole workgroup
  const uint32_t c = cb * kInferThreads + threadIdx.x;
  const bool col_ok = c < sh.C;
  const uint32_t n = col_ok ? cnt[c] : 0u;
  const uint32_t f0 = fg * frames_per_group;
  const uint32_t f1 = min(F, f0 + frames_per_group);
  for (uint32_t f = f0; f < f1; ++f) {
    const uint32_t* frame = frames + (size_t)f * sh.W;
    if constexpr (LDS) {
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < sh.W; i += kInferThreads) fr[i] = frame[i];
      __syncthreads();
    }
    uint32_t acc = 0;
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t e = list[(size_t)i * sh.C + c];
      const uint32_t word = LDS ? entry_load(fr, e) : frame[entry_word(e)];
      acc += __builtin_amdgcn_ubfe(word, e, 1);
    }
    if (col_ok) ov_out[(size_t)f * sh.C + c] = acc >= sh.m ? (int32_t)acc : 0;
  }
}

// Gather overlaps with two frame buffers in LDS: while the workgroup counts
// frame f from one buffer, frame f + 1 streams into the other with direct
// global-to-LDS loads (no registers, no wait until the end of frame f).
// One workgroup per CU (two 960x540 frames take 130 KB of LDS), THREADS
// columns per workgroup; block ids map to (frame group, column block) as in
// k_infer_gather.  The buffers sit at fixed LDS offsets so that the second
// one is an immediate offset of the read.  `vec`: frames are 16-byte aligned
// rows, so whole rows move in 16-byte pieces.
constexpr uint32_t kDbBufWords = 16256;  // 65 024 B: the largest immediate-offset buffer

template <int MAXN, int THREADS>
__global__ __launch_bounds__(THREADS) void k_infer_gather_db(
    const uint32_t* __restrict__ frames, uint32_t F, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ cnt, Shape sh, uint32_t frames_per_group, uint32_t col_blocks,
    uint32_t groups, int32_t* __restrict__ ov_out, uint32_t vec) {
  __shared__ uint32_t lds[2 * kDbBufWords];
  const uint32_t per = 8 * col_blocks;
  const uint32_t fg = (blockIdx.x / per) * 8 + blockIdx.x % 8;
  const uint32_t cb = (blockIdx.x % per) / 8;
  if (fg >= groups) return;  // whole workgroup
  const uint32_t tid = threadIdx.x, lane = tid % kWave;
  const uint32_t c = cb * THREADS + tid;
  const bool col_ok = c < sh.C;
  const uint32_t pad = sh.W << 7;

  uint32_t lst[MAXN];
#pragma unroll
  for (int i = 0; i < MAXN; ++i)
    lst[i] = (col_ok && (uint32_t)i < sh.S) ? list[(size_t)i * sh.C + c] : pad;
  uint32_t n = col_ok ? cnt[c] : 0u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n = max(n, (uint32_t)__shfl_xor(n, off));

  // Frame f into buffer b: the LDS address of a direct load is the wave's
  // base plus the lane's offset, so the base passed is that of lane 0.
  auto stage = [&](uint32_t f, uint32_t b) {
    const uint32_t* fr = frames + (size_t)f * sh.W;
    uint32_t* dst = lds + b * kDbBufWords;
    if (vec) {
      const uint32_t n4 = sh.W / 4;
      for (uint32_t i = tid; i < n4; i += THREADS)
        __builtin_amdgcn_global_load_lds(fr + 4 * i, dst + 4 * (i - lane), 16, 0, 0);
    } else {
      for (uint32_t i = tid; i < sh.W; i += THREADS)
        __builtin_amdgcn_global_load_lds(fr + i, dst + (i - lane), 4, 0, 0);
    }
  };
  // Counts frame f from buffer B, prefetching frame f + 1 into the other.
  const uint32_t f0 = fg * frames_per_group;
  const uint32_t f1 = min(F, f0 + frames_per_group);
  auto frame = [&](uint32_t f, auto B) {
    constexpr uint32_t b = decltype(B)::value;
    if (f + 1 < f1) stage(f + 1, b ^ 1u);
    const uint32_t* fr = lds + b * kDbBufWords;
    // one register per list entry (see k_infer_gather)
#pragma unroll
    for (int i = 0; i < MAXN; ++i) asm volatile("" : "+v"(lst[i]));
    uint32_t acc = 0;
#pragma unroll
    for (int i0 = 0; i0 < MAXN; i0 += 16) {
      if ((uint32_t)i0 < n) {
#pragma unroll
        for (int i = i0; i < i0 + 16; ++i) {
          const uint32_t e = lst[i];
          acc += __builtin_amdgcn_ubfe(entry_load(fr, e), e, 1);
        }
      }
    }
    if (col_ok) ov_out[(size_t)f * sh.C + c] = acc >= sh.m ? (int32_t)acc : 0;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };

  if (tid == 0) {
    lds[sh.W] = 0u;  // the padding entry's word, in both buffers
    lds[kDbBufWords + sh.W] = 0u;
  }
  stage(f0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (uint32_t f = f0; f < f1; f += 2) {
    frame(f, std::integral_constant<uint32_t, 0>());
    if (f + 1 < f1) frame(f + 1, std::integral_constant<uint32_t, 1>());
  }
}

// Global top-k of each frame (one wave per frame): overlaps packed four per
// 64-bit word, the threshold by count probes, winners compacted in column
// order, -1 padding.
template <int NV>
__global__ __launch_bounds__(256) void k_topk_batch(const int32_t* __restrict__ ov, uint32_t F,
                                                    Shape sh, int32_t* __restrict__ winners) {
  const uint32_t f = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x % kWave;
  if (f >= F) return;
  const int32_t* o = ov + (size_t)f * sh.C;
  uint64_t ev[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    uint64_t w = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t c = (uint32_t)u * 4 * kWave + 4 * lane + q;
      const uint32_t v = c < sh.C ? (uint32_t)o[c] : 0u;
      w |= (uint64_t)v << (16 * q);
    }
    ev[u] = w;
  }
  uint32_t c_hi;
  const uint32_t T = topk_threshold(ev, sh.S, sh.k, 1 + sh.S / 16, &c_hi);
  const uint32_t need = T ? sh.k - c_hi : 0u;
  const uint32_t nsel = T ? sh.k : c_hi;
  uint64_t fm[NV];
  select_all(ev, T, need, lane, fm);
  int32_t* wrow = winners + (size_t)f * sh.k;
  uint32_t base = 0;
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const uint64_t sel = fm[u] & kHighBits;
    const uint32_t n = (uint32_t)__popcll(sel);
    uint32_t pos = base + wave_prefix<3>(n, lane);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      if (sel & (0x8000ull << (16 * q))) {
        wrow[pos] = (int32_t)((uint32_t)u * 4 * kWave + 4 * lane + q);
        ++pos;
      }
    }
    base += wave_count<3>(n);
  }
  for (uint32_t i = nsel + lane; i < sh.k; i += kWave) wrow[i] = -1;
}

template <int MAXN, bool LDS>
hipError_t launch_gather_t(const uint32_t* frames, uint32_t F, const uint32_t* list,
                           const uint32_t* cnt, const Shape& sh, int32_t* ov, uint32_t cus,
                           hipStream_t s) {
  const uint32_t col_blocks = (sh.C + kInferThreads - 1) / kInferThreads;
  // about two blocks per CU, frame groups a multiple of 8
  uint32_t groups = (2 * cus + col_blocks - 1) / col_blocks;
  groups = min(groups, F);
  const uint32_t fpg = (F + groups - 1) / groups;
  groups = (F + fpg - 1) / fpg;
  const uint32_t padded = (groups + 7) / 8 * 8;
  const size_t lds = LDS ? sizeof(uint32_t) * ((size_t)sh.W + 1) : 0;
  hipLaunchKernelGGL((k_infer_gather<MAXN, LDS>), dim3(padded * col_blocks), dim3(kInferThreads),
                     lds, s, frames, F, list, cnt, sh, fpg, col_blocks, groups, ov);
  return hipGetLastError();
}

template <bool LDS>
hipError_t launch_gather_l(uint32_t maxn, const uint32_t* frames, uint32_t F,
                           const uint32_t* list, const uint32_t* cnt, const Shape& sh,
                           int32_t* ov, uint32_t cus, hipStream_t s) {
  if (maxn <= 32) return launch_gather_t<32, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  if (maxn <= 64) return launch_gather_t<64, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  if (maxn <= 96) return launch_gather_t<96, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  if (maxn <= 128) return launch_gather_t<128, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  if (maxn <= 160) return launch_gather_t<160, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  if (maxn <= 192) return launch_gather_t<192, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  if (maxn <= 224) return launch_gather_t<224, LDS>(frames, F, list, cnt, sh, ov, cus, s);
  return launch_gather_t<256, LDS>(frames, F, list, cnt, sh, ov, cus, s);
}

template <int MAXN, int THREADS>
hipError_t launch_gather_db_t(const uint32_t* frames, uint32_t F, const uint32_t* list,
                              const uint32_t* cnt, const Shape& sh, int32_t* ov, uint32_t cus,
                              hipStream_t s) {
  const uint32_t col_blocks = (sh.C + THREADS - 1) / THREADS;
  // one workgroup per CU, frame groups a multiple of 8
  uint32_t groups = (cus + col_blocks - 1) / col_blocks;
  groups = max(1u, min(groups, F));
  const uint32_t fpg = (F + groups - 1) / groups;
  groups = (F + fpg - 1) / fpg;
  const uint32_t padded = (groups + 7) / 8 * 8;
  const uint32_t vec = ((reinterpret_cast<uintptr_t>(frames) & 15u) == 0 && sh.W % 4 == 0);
  hipLaunchKernelGGL((k_infer_gather_db<MAXN, THREADS>), dim3(padded * col_blocks),
                     dim3(THREADS), 0, s, frames, F, list, cnt, sh, fpg, col_blocks, groups,
                     ov, vec);
  return hipGetLastError();
}

template <bool LDS>
hipError_t launch_gather_long_t(const uint32_t* frames, uint32_t F, const uint32_t* list,
                                const uint32_t* cnt, const Shape& sh, int32_t* ov, uint32_t cus,
                                hipStream_t s) {
  const uint32_t col_blocks = (sh.C + kInferThreads - 1) / kInferThreads;
  // about four blocks per CU, frame groups a multiple of 8
  uint32_t groups = (4 * cus + col_blocks - 1) / col_blocks;
  groups = max(1u, min(groups, F));
  const uint32_t fpg = (F + groups - 1) / groups;
  groups = (F + fpg - 1) / fpg;
  const uint32_t padded = (groups + 7) / 8 * 8;
  const size_t lds = LDS ? sizeof(uint32_t) * (size_t)sh.W : 0;
  hipLaunchKernelGGL((k_infer_gather_long<LDS>), dim3(padded * col_blocks), dim3(kInferThreads),
                     lds, s, frames, F, list, cnt, sh, fpg, col_blocks, groups, ov);
  return hipGetLastError();
}

hipError_t launch_gather_db(uint32_t maxn, const uint32_t* frames, uint32_t F,
                            const uint32_t* list, const uint32_t* cnt, const Shape& sh,
                            int32_t* ov, uint32_t cus, hipStream_t s) {
#define HTMSP_DB(M, T) \
  if (maxn <= M) return launch_gather_db_t<M, T>(frames, F, list, cnt, sh, ov, cus, s);
  HTMSP_DB(32, 512) HTMSP_DB(64, 512) HTMSP_DB(96, 512) HTMSP_DB(128, 512)
  HTMSP_DB(160, 512) HTMSP_DB(192, 512) HTMSP_DB(224, 256)
#undef HTMSP_DB
  return launch_gather_db_t<256, 256>(frames, F, list, cnt, sh, ov, cus, s);
}

}  // namespace

uint32_t infer_max_list() { return 256; }

size_t infer_lds_limit() { return 65536; }

hipError_t launch_infer_prep(const uint32_t* idx, const float* perm, const Shape& sh,
                             uint32_t* list, uint32_t* cnt, uint32_t* maxcnt, hipStream_t s) {
  if (maxcnt) {
    hipError_t e = hipMemsetAsync(maxcnt, 0, sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_infer_prep, dim3((sh.C + 255) / 256), dim3(256), 0, s, idx, perm, sh,
                     sh.W << 7, list, cnt, maxcnt);
  return hipGetLastError();
}

hipError_t launch_infer_gather(uint32_t maxn, const uint32_t* frames, uint32_t F,
                               const uint32_t* list, const uint32_t* cnt, const Shape& sh,
                               int32_t* ov, uint32_t cus, hipStream_t s) {
  int dev = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  if (maxn > infer_max_list()) {
    // every entry is a real connected input (no padding read), so the frame
    // needs no zero word
    const bool lds = sizeof(uint32_t) * (size_t)sh.W <= infer_lds_limit();
    return lds ? launch_gather_long_t<true>(frames, F, list, cnt, sh, ov, cus, s)
               : launch_gather_long_t<false>(frames, F, list, cnt, sh, ov, cus, s);
  }
  // two buffers, each the frame plus the zero word
  if (sh.W + 1 <= kDbBufWords && sizeof(uint32_t) * 2 * kDbBufWords <= (size_t)lds_max)
    return launch_gather_db(maxn, frames, F, list, cnt, sh, ov, cus, s);
  const bool lds = sizeof(uint32_t) * ((size_t)sh.W + 1) <= infer_lds_limit();
  return lds ? launch_gather_l<true>(maxn, frames, F, list, cnt, sh, ov, cus, s)
             : launch_gather_l<false>(maxn, frames, F, list, cnt, sh, ov, cus, s);
}

hipError_t launch_topk_batch(const int32_t* ov, uint32_t F, const Shape& sh, int32_t* winners,
                             hipStream_t s) {
  const uint32_t blocks = (F + 3) / 4;
  const uint32_t nv = (sh.C + 255) / 256;
#define HTMSP_TB(V)                                                                         \
  if (nv <= V) {                                                                            \
    hipLaunchKernelGGL(k_topk_batch<V>, dim3(blocks), dim3(256), 0, s, ov, F, sh, winners); \
    return hipGetLastError();                                                               \
  }
  HTMSP_TB(1) HTMSP_TB(2) HTMSP_TB(4) HTMSP_TB(8) HTMSP_TB(16)
#undef HTMSP_TB
  return hipErrorInvalidValue;
}

}  // namespace htmsp
