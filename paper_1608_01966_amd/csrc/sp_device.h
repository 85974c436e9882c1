// Device helpers shared by the spatial pooler kernels (sp_kernels.hip,
// sp_infer.hip).  Not part of the ABI.
//
// Permanences are handled as integers q = 256 * permanence (0..256), so every
// comparison and update is exact.  Overlaps of a frame are often held packed,
// four 14-bit values per 64-bit word (16-bit fields); word u of lane l then
// holds columns u*256 + 4*l + {0, 1, 2, 3}.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sp_internal.h"

namespace htmsp {
namespace dev {

constexpr uint32_t kWave = 64;

__device__ __forceinline__ uint32_t perm_to_q(float p) {
  int q = (int)(p * 256.0f);
  return (uint32_t)min(max(q, 0), 256);
}

__device__ __forceinline__ float q_to_perm(uint32_t q) { return (float)q * (1.0f / 256.0f); }

__device__ __forceinline__ uint32_t input_bit(uint32_t word, uint32_t i) {
  return (word >> (i & 31u)) & 1u;
}

__device__ __forceinline__ uint32_t learn_q(uint32_t q, uint32_t bit, const Shape& sh) {
  return bit ? min(q + sh.inc, 256u) : (uint32_t)max((int)q - (int)sh.dec, 0);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint64_t lanemask_lt(uint32_t lane) { return (1ull << lane) - 1ull; }

__device__ __forceinline__ uint32_t load_tagged(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_tagged(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Packed 16-bit fields: [tag:2 | value:14].
constexpr uint32_t kTagShift = 14;
constexpr uint64_t kFieldBits = 0x3FFF3FFF3FFF3FFFull;
constexpr uint64_t kTagBits = 0xC000C000C000C000ull;
constexpr uint64_t kHighBits = 0x8000800080008000ull;
constexpr uint64_t kOnes16 = 0x0001000100010001ull;

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

__device__ __forceinline__ uint32_t lds_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// c added to each of the four 16-bit fields of w, where no field sum
// reaches 2^16: nothing carries between fields, so the two 32-bit halves add
// on their own (two full-rate adds, not a 64-bit multiply-add).
__device__ __forceinline__ uint64_t field_add(uint64_t w, uint32_t c) {
  const uint32_t cc = c * 0x10001u;
  return ((uint64_t)((uint32_t)(w >> 32) + cc) << 32) | (uint32_t)((uint32_t)w + cc);
}

// Fields of w (four 16-bit fields holding values < 2^14) that are >= x,
// for 1 <= x <= 2^14: field + 0x8000 - x reaches bit 15 exactly when
// field >= x, and never carries into the next field.
__device__ __forceinline__ uint32_t fields_ge(uint64_t w, uint32_t x, uint64_t keep) {
  return (uint32_t)__popcll(field_add(w, 0x8000u - x) & keep);
}

// Sum over the wave of per-lane counts below 2^BITS, one ballot per bit.
template <int BITS>
__device__ __forceinline__ uint32_t wave_count(uint32_t v) {
  uint32_t s = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) s += (uint32_t)__popcll(__ballot((v >> b) & 1u)) << b;
  return s;
}

// Columns (all, or only those below c_end) whose overlap is >= x.  Word u
// of this lane holds columns u*256 + 4*lane + {0, 1, 2, 3}.
template <int NV>
__device__ __forceinline__ uint32_t count_ge(const uint64_t (&ev)[NV], uint32_t x) {
  uint32_t n = 0;
#pragma unroll
  for (int u = 0; u < NV; ++u) n += fields_ge(ev[u], x, kHighBits);
  return wave_count<ilog2(4 * NV) + 1>(n);
}

template <int NV>
__device__ __forceinline__ uint32_t count_ge_before(const uint64_t (&ev)[NV], uint32_t x,
                                                    uint32_t lane, uint32_t c_end) {
  uint32_t n = 0;
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const uint32_t cb = (uint32_t)u * 4 * kWave + 4 * lane;
    const uint32_t nin = c_end > cb ? min(4u, c_end - cb) : 0u;
    const uint64_t keep = nin >= 4 ? kHighBits : (((1ull << (16 * nin)) - 1ull) & kHighBits);
    n += fields_ge(ev[u], x, keep);
  }
  return wave_count<ilog2(4 * NV) + 1>(n);
}

// Columns below c_end whose overlap equals x (1 <= x < 2^14): fields >= x
// and not >= x + 1, counted in one wave sum.
template <int NV>
__device__ __forceinline__ uint32_t count_eq_before(const uint64_t (&ev)[NV], uint32_t x,
                                                    uint32_t lane, uint32_t c_end) {
  uint32_t n = 0;
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const uint32_t cb = (uint32_t)u * 4 * kWave + 4 * lane;
    const uint32_t nin = c_end > cb ? min(4u, c_end - cb) : 0u;
    const uint64_t keep = nin >= 4 ? kHighBits : (((1ull << (16 * nin)) - 1ull) & kHighBits);
    const uint64_t ge = field_add(ev[u], 0x8000u - x);
    const uint64_t gt = field_add(ev[u], 0x7FFFu - x);
    n += (uint32_t)__popcll(ge & ~gt & keep);
  }
  return wave_count<ilog2(4 * NV) + 1>(n);
}

// Exclusive prefix over lanes of per-lane counts below 2^BITS.
template <int BITS>
__device__ __forceinline__ uint32_t wave_prefix(uint32_t v, uint32_t lane) {
  const uint64_t lt = lanemask_lt(lane);
  uint32_t s = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) s += (uint32_t)__popcll(__ballot((v >> b) & 1u) & lt) << b;
  return s;
}

// Field masks of the winners among all columns of one frame: every field
// above T, and the first `need` fields equal to T in column order (word u,
// lane l, field q is column u*256 + 4*l + q).  T == 0 selects every
// positive field.  T and need are the same in every lane, so the words
// before the one where the ties run out take all their ties, the words after
// it none, and only that one word ranks its ties across the wave.  Within a
// lane, (eq >> 15) * kOnes16 holds in each field the number of tied fields up
// to and including it, which the field-wise compare keeps to `keep`.
template <int NV>
__device__ __forceinline__ void select_all(const uint64_t (&ev)[NV], uint32_t T, uint32_t need,
                                           uint32_t lane, uint64_t (&fm)[NV]) {
  T = __builtin_amdgcn_readfirstlane(T);
  need = __builtin_amdgcn_readfirstlane(need);
  uint32_t before = 0;  // fields equal to T in earlier words, whole wave
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const uint64_t gt = field_add(ev[u], 0x7FFFu - T) & kHighBits;
    uint64_t take = 0;
    if (T != 0 && before < need) {
      const uint64_t eq = (field_add(ev[u], 0x8000u - T) & kHighBits) & ~gt;
      const uint32_t n = (uint32_t)__popcll(eq);
      const uint32_t tot = wave_count<3>(n);
      if (before + tot <= need) {
        take = eq;
      } else {
        const uint32_t pre = before + wave_prefix<3>(n, lane);
        const uint32_t keep = need > pre ? min(need - pre, 4u) : 0u;
        const uint64_t cum = (eq >> 15) * kOnes16;
        take = eq & ~(field_add(cum, 0x7FFFu - keep) & kHighBits);
      }
      before += tot;
    }
    fm[u] = ((gt | take) >> 15) * 0xFFFFull;
  }
}

// Global top-k threshold (Algorithm 2, global form): T = the largest x >= 1
// with #(overlap >= x) >= k, or 0 when fewer than k overlaps are positive;
// *c_hi = #(overlap >= T + 1).  Invariant: #(overlap >= lo) >= k unless
// lo == 0, and c_hi = #(overlap >= hi + 1) < k.  A gallop from `guess`
// narrows [lo, hi], a binary search finishes it.
template <int NV>
__device__ __forceinline__ uint32_t topk_threshold(const uint64_t (&ev)[NV], uint32_t S,
                                                   uint32_t k, uint32_t guess, uint32_t* c_hi_out) {
  uint32_t lo = 0, hi = S, c_hi = 0;
  const uint32_t g0 = min(max(guess, 1u), S);
  const uint32_t c0 = count_ge(ev, g0);
  if (c0 >= k) {
    lo = g0;
    for (uint32_t step = 1; lo < hi; step <<= 1) {
      const uint32_t x = min(lo + step, hi);
      const uint32_t cx = count_ge(ev, x);
      if (cx >= k) {
        lo = x;
      } else {
        hi = x - 1;
        c_hi = cx;
        break;
      }
    }
  } else {
    hi = g0 - 1;
    c_hi = c0;
    for (uint32_t step = 1; hi > 0; step <<= 1) {
      const uint32_t x = hi >= step ? hi - step + 1 : 1u;
      const uint32_t cx = count_ge(ev, x);
      if (cx >= k) {
        lo = x;
        break;
      }
      hi = x - 1;
      c_hi = cx;
    }
  }
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    const uint32_t c = count_ge(ev, mid);
    if (c >= k) {
      lo = mid;
    } else {
      hi = mid - 1;
      c_hi = c;
    }
  }
  *c_hi_out = c_hi;
  return lo;
}

// ---- Persistent exchanges between workgroups ----
__device__ __forceinline__ void lds_release(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Agent-scope 64-bit store and load of four packed exchange entries.
__device__ __forceinline__ void store_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_entries(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Element `lane` of a wave-uniform array, in lane `lane` (0 past CPW).
template <int CPW>
__device__ __forceinline__ uint32_t lane_value(const uint32_t (&ovs)[CPW], uint32_t lane) {
  uint32_t v = 0;
#pragma unroll
  for (uint32_t j = 0; j < (uint32_t)CPW; ++j) v = lane == j ? ovs[j] : v;
  return v;
}

// The XCD this wave runs on.
__device__ __forceinline__ uint32_t xcc_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v;
}

// Tag bits to check in exchange word u of this lane, whose entries are
// columns u * 256 + 4 * lane + {0..3} (entries at or past C are never
// written and are skipped).
__device__ __forceinline__ uint64_t tag_mask(uint32_t u, uint32_t lane, uint32_t C) {
  const uint32_t cb = u * 4 * kWave + 4 * lane;
  if (cb + 4 <= C) return kTagBits;
  const uint32_t n = C > cb ? C - cb : 0u;
  return ((1ull << (16 * n)) - 1ull) & kTagBits;
}

}  // namespace dev
}  // namespace htmsp
