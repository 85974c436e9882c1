// Batched inference as a dense int8 matrix product (Section 4.1's testing
// mode, learning off; overlap as in Algorithm 1, a column's count of
// connected synapses whose input bit is on):
//
//   raw[f][c] = sum over pixels n of X[f][n] * M[n][c]
//
// with X[f][n] the 0/1 input bit of frame f and M[n][c] = 1 when column c has
// a connected synapse on pixel n.  Both operands stay bit-packed in device
// memory (the frames as the caller passes them, the mask as [C][Wm] words
// built once per state version) and are widened to int8 0/1 in registers
// right before each v_mfma_i32_16x16x64_i8, which accumulates exactly in
// int32.  The gate (min_overlap) is the epilogue; the global top-k of each
// frame is the batched top-k of the gather form.
//
// Widening: a 32-bit word x of 32 pixels gives eight 4-byte groups
// (x >> r) & 0x01010101, r = 0..7, group r holding pixels r, 8 + r, 16 + r,
// 24 + r.  The contraction runs over pixels in that order inside each
// 512-pixel block; it is the same order for both operands, so each product
// pairs the same pixel of the frame and of the mask.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr uint32_t kMfThreads = 256;  // four independent waves
constexpr uint32_t kMfRowBlocks = 4;  // 16-frame blocks per wave tile (64 frames)
constexpr uint32_t kMfColBlocks = 8;  // 16-column blocks per wave tile (128 columns)
constexpr uint32_t kMfTileF = 16 * kMfRowBlocks;
constexpr uint32_t kMfTileC = 16 * kMfColBlocks;
constexpr uint32_t kMfBlockWords = 16;  // words per 512-pixel block: 8 steps of 64 pixels

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Connected mask of column c as bits over the pixels (row c of [C][Wm]
// words, zeroed beforehand); *dup counts connected synapses that land on a
// pixel another connected synapse of the same column already set (the 0/1
// mask cannot hold a count of 2).
__global__ __launch_bounds__(256) void k_mfma_mask(const uint32_t* __restrict__ idx,
                                                   const float* __restrict__ perm, Shape sh,
                                                   uint32_t Wm, uint32_t* __restrict__ mask,
                                                   uint32_t* __restrict__ dup) {
  const size_t n = (size_t)sh.C * sh.S;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    if (dev::perm_to_q(perm[i]) < sh.theta) continue;
    const uint32_t c = (uint32_t)(i / sh.S);
    const uint32_t p = min(idx[i], sh.N - 1);
    const uint32_t bit = 1u << (p & 31u);
    const uint32_t old = atomicOr(&mask[(size_t)c * Wm + (p >> 5)], bit);
    if (old & bit) atomicAdd(dup, 1u);
  }
}

struct MfmaArgs {
  const uint32_t* frames;  // [F][W]
  const uint32_t* mask;    // [C][Wm], Wm a multiple of kMfBlockWords, zero past W
  int32_t* out;            // splits == 1: gated overlaps [F][C]; else partial sums [splits][F][C]
  uint32_t F, C, W, Wm, m;
  uint32_t tiles_f, tiles_c, splits, blocks_per_split;
  uint32_t full_blocks;    // 512-pixel blocks lying wholly inside a frame row (W / 16)
  uint32_t nblocks;        // Wm / 16
  uint32_t units;          // wave tiles: splits * tiles_f * tiles_c
  uint32_t per_xcd;        // wave tiles per XCD (a multiple of 4)
  uint32_t vec;            // frame rows are 16-byte aligned
};

// The four bytes of group r of x, widened: pixels r, 8 + r, 16 + r, 24 + r.
__device__ __forceinline__ int widen(uint32_t x, uint32_t r) {
  return (int)((x >> r) & 0x01010101u);
}

__device__ __forceinline__ uint32_t word_of(const uint4& v, uint32_t j) {
  return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w;
}

// The eight 64-pixel steps of one 512-pixel block: step s uses word s / 2
// of each lane's four and groups 4 (s % 2) .. 4 (s % 2) + 3 of it.
__device__ __forceinline__ void mfma_block(const uint4 (&xa)[kMfRowBlocks],
                                           const uint4 (&xb)[kMfColBlocks],
                                           v4i (&acc)[kMfRowBlocks][kMfColBlocks]) {
#pragma unroll
  for (uint32_t s = 0; s < 8; ++s) {
    const uint32_t j = s / 2, r0 = 4 * (s % 2);
    v4i fa[kMfRowBlocks], fb[kMfColBlocks];
#pragma unroll
    for (uint32_t r = 0; r < kMfRowBlocks; ++r) {
      const uint32_t x = word_of(xa[r], j);
      fa[r] = v4i{widen(x, r0), widen(x, r0 + 1), widen(x, r0 + 2), widen(x, r0 + 3)};
    }
#pragma unroll
    for (uint32_t c = 0; c < kMfColBlocks; ++c) {
      const uint32_t x = word_of(xb[c], j);
      fb[c] = v4i{widen(x, r0), widen(x, r0 + 1), widen(x, r0 + 2), widen(x, r0 + 3)};
    }
#pragma unroll
    for (uint32_t r = 0; r < kMfRowBlocks; ++r)
#pragma unroll
      for (uint32_t c = 0; c < kMfColBlocks; ++c)
        acc[r][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[r], fb[c], acc[r][c], 0, 0, 0);
  }
}

// One wave computes a 64-frame x 128-column tile over the 512-pixel blocks of
// its split.  Lane (i, g) = (lane % 16, lane / 16) holds rows i of every
// 16-row block and words 4g .. 4g + 3 of each 512-pixel block; step s (0..7)
// of a block uses word s / 2 and groups 4 (s % 2) .. 4 (s % 2) + 3 of it, for
// the frames and for the mask alike.  VEC: frame rows are 16-byte aligned
// (16-byte loads).  Wave tiles are dealt to XCDs in
// contiguous runs (block b runs on XCD b % 8), so the waves that share frames
// and mask rows share an L2.
template <bool VEC>
__global__ __launch_bounds__(kMfThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_infer_mfma(MfmaArgs a) {
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t slot = (blockIdx.x / 8) * 4 + wv;
  if (slot >= a.per_xcd) return;
  const uint32_t u = (blockIdx.x % 8) * a.per_xcd + slot;
  if (u >= a.units) return;
  const uint32_t tc = u % a.tiles_c, rest = u / a.tiles_c;
  const uint32_t tf = rest % a.tiles_f, split = rest / a.tiles_f;
  const uint32_t b0 = split * a.blocks_per_split;
  const uint32_t b1 = min(a.nblocks, b0 + a.blocks_per_split);
  const uint32_t i16 = lane & 15u, g = lane >> 4;

  // Word offsets of this lane's rows (the host keeps F * W and C * Wm below
  // 2^31); rows past F or C repeat the last one, and their sums are not
  // stored.
  uint32_t arow[kMfRowBlocks], brow[kMfColBlocks];
#pragma unroll
  for (uint32_t r = 0; r < kMfRowBlocks; ++r)
    arow[r] = min(tf * kMfTileF + 16 * r + i16, a.F - 1) * a.W + 4 * g;
#pragma unroll
  for (uint32_t c = 0; c < kMfColBlocks; ++c)
    brow[c] = min(tc * kMfTileC + 16 * c + i16, a.C - 1) * a.Wm + 4 * g;

  v4i acc[kMfRowBlocks][kMfColBlocks];
#pragma unroll
  for (uint32_t r = 0; r < kMfRowBlocks; ++r)
#pragma unroll
    for (uint32_t c = 0; c < kMfColBlocks; ++c) acc[r][c] = v4i{0, 0, 0, 0};

  for (uint32_t blk = b0; blk < b1; ++blk) {
    const uint32_t wbase = blk * kMfBlockWords;
    uint4 xa[kMfRowBlocks], xb[kMfColBlocks];
#pragma unroll
    for (uint32_t c = 0; c < kMfColBlocks; ++c)
      xb[c] = *reinterpret_cast<const uint4*>(a.mask + (brow[c] + wbase));
    if (blk < a.full_blocks) {
#pragma unroll
      for (uint32_t r = 0; r < kMfRowBlocks; ++r) {
        const uint32_t* p = a.frames + (arow[r] + wbase);
        if constexpr (VEC) {
          xa[r] = *reinterpret_cast<const uint4*>(p);
        } else {
          xa[r] = uint4{p[0], p[1], p[2], p[3]};
        }
      }
    } else {
      // the last block of a row: words at or past W read as 0
      const uint32_t w0 = wbase + 4 * g;
#pragma unroll
      for (uint32_t r = 0; r < kMfRowBlocks; ++r) {
        const uint32_t* p = a.frames + (arow[r] + wbase);
        xa[r] = uint4{w0 + 0 < a.W ? p[0] : 0u, w0 + 1 < a.W ? p[1] : 0u,
                      w0 + 2 < a.W ? p[2] : 0u, w0 + 3 < a.W ? p[3] : 0u};
      }
    }
    mfma_block(xa, xb, acc);
  }

  // Lane (i, g), register q of block (r, c) holds frame 16 r + 4 g + q and
  // column 16 c + i of the tile.
  int32_t* out = a.out + (size_t)split * a.F * a.C;
#pragma unroll
  for (uint32_t r = 0; r < kMfRowBlocks; ++r) {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t f = tf * kMfTileF + 16 * r + 4 * g + q;
      if (f >= a.F) continue;
#pragma unroll
      for (uint32_t c = 0; c < kMfColBlocks; ++c) {
        const uint32_t col = tc * kMfTileC + 16 * c + i16;
        if (col >= a.C) continue;
        int32_t v = acc[r][c][q];
        if (a.splits == 1) v = (uint32_t)v >= a.m ? v : 0;
        out[(size_t)f * a.C + col] = v;
      }
    }
  }
}

// Sums the partial products of the splits and applies the min_overlap gate.
__global__ __launch_bounds__(256) void k_mfma_reduce(const int32_t* __restrict__ part,
                                                     uint32_t splits, size_t n, uint32_t m,
                                                     int32_t* __restrict__ ov) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (uint32_t s = 0; s < splits; ++s) v += (uint32_t)part[(size_t)s * n + i];
    ov[i] = v >= m ? (int32_t)v : 0;
  }
}

uint32_t grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  return (uint32_t)std::max<size_t>(1, std::min<size_t>(b, 4096));
}

}  // namespace

uint32_t mfma_mask_words(uint32_t W) {
  return (W + kMfBlockWords - 1) / kMfBlockWords * kMfBlockWords;
}

hipError_t launch_mfma_mask(const uint32_t* idx, const float* perm, const Shape& sh,
                            uint32_t* mask, uint32_t* dup, hipStream_t s) {
  const uint32_t Wm = mfma_mask_words(sh.W);
  const size_t words = (size_t)sh.C * Wm;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words)), dim3(256), 0, s, mask, words, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, dup, (size_t)1, 0u);
  hipLaunchKernelGGL(k_mfma_mask, dim3(grid_for((size_t)sh.C * sh.S)), dim3(256), 0, s, idx,
                     perm, sh, Wm, mask, dup);
  return hipGetLastError();
}

uint32_t mfma_splits(const Shape& sh, uint32_t F, uint32_t cus) {
  const uint32_t nblocks = mfma_mask_words(sh.W) / kMfBlockWords;
  const size_t tiles = (size_t)((F + kMfTileF - 1) / kMfTileF) * ((sh.C + kMfTileC - 1) / kMfTileC);
  // two waves per SIMD fill the device (the kernel holds 2 of its
  // workgroups per CU)
  const size_t target = (size_t)cus * 8;
  uint32_t splits = (uint32_t)std::min<size_t>(8, (target + tiles - 1) / tiles);
  splits = std::max(1u, std::min(splits, nblocks));
  const uint32_t per = (nblocks + splits - 1) / splits;
  return (nblocks + per - 1) / per;
}

hipError_t launch_infer_mfma(const uint32_t* frames, uint32_t F, const uint32_t* mask,
                             const Shape& sh, uint32_t splits, int32_t* part, int32_t* ov,
                             hipStream_t s) {
  MfmaArgs a;
  a.frames = frames;
  a.mask = mask;
  a.F = F;
  a.C = sh.C;
  a.W = sh.W;
  a.Wm = mfma_mask_words(sh.W);
  a.m = sh.m;
  a.tiles_f = (F + kMfTileF - 1) / kMfTileF;
  a.tiles_c = (sh.C + kMfTileC - 1) / kMfTileC;
  a.nblocks = a.Wm / kMfBlockWords;
  a.full_blocks = sh.W / kMfBlockWords;
  a.blocks_per_split = (a.nblocks + splits - 1) / splits;
  a.splits = (a.nblocks + a.blocks_per_split - 1) / a.blocks_per_split;
  a.out = a.splits == 1 ? ov : part;
  a.units = a.splits * a.tiles_f * a.tiles_c;
  a.per_xcd = ((a.units + 7) / 8 + 3) / 4 * 4;
  a.vec = ((reinterpret_cast<uintptr_t>(frames) & 15u) == 0 && sh.W % 4 == 0) ? 1u : 0u;
  const uint32_t blocks = 8 * (a.per_xcd / 4);
  if (a.vec)
    hipLaunchKernelGGL(k_infer_mfma<true>, dim3(blocks), dim3(kMfThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_infer_mfma<false>, dim3(blocks), dim3(kMfThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.splits == 1) return e;
  const size_t n = (size_t)F * sh.C;
  hipLaunchKernelGGL(k_mfma_reduce, dim3(grid_for(n)), dim3(256), 0, s, part, a.splits, n, sh.m,
                     ov);
  return hipGetLastError();
}

}  // namespace htmsp
