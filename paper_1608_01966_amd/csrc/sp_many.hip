// Many independent spatial pooler instances stepped by one persistent
// launch (Section 3.1's 'Multiple HTMs' setup runs one pooler per category;
// serving runs one per video stream).  Each instance still follows Section
// 1.1 frame by frame -- overlap, global inhibition, learning -- so its frames
// are sequential, but the instances are independent: while one waits for its
// inhibition, the GPU works on the others.
//
// Work is split into tasks, assigned statically to the workgroups of a
// cooperative grid (tile workgroups first, then top-k workgroups):
//   tile task (instance, columns [c0, c1)), at most kTileSynapses synapses,
//     the whole workgroup: once the instance's decision of step t-1 is out,
//     its step t applies learning of frame t-1 to its winning columns, then
//     computes the overlaps of frame t and publishes them.  Each thread owns
//     up to 16 synapses of the tile's flat [column][synapse] range and issues
//     all their state loads, then both input gathers, at once; per-column
//     counts are summed in LDS, and each tile keeps its last published
//     overlaps in LDS to decide its winners.  A workgroup steps whichever of
//     its tiles is ready.
//   top-k task (instance), one wave: for step t it collects the instance's
//     overlaps, resolves the global top-k, writes the frame's outputs (and
//     adds the winners to the instance's histogram, if it has one) and
//     publishes a decision word from which every tile derives which of its
//     columns won.
// Synapse state is read from and written to device memory every step (the
// instances' state does not fit on chip together).  Every cross-workgroup
// value carries its step's tag (overlap entries [tag:16 | overlap:16],
// decision [tag:16 | T:16 | last tied winner + 1:32]) and is written and read
// with agent-scope atomics, so no fence is needed; a tag never matches a
// value left by an earlier step, and an instance's buffers are rewritten only
// after their readers are done with them (tiles wait for the previous
// decision, which the top-k task publishes after reading every overlap).
// Aborts (spin limit, error word) are made uniform over the workgroup before
// its next barrier, so a failing launch still drains.
#include "sp_device.h"
#include "sp_internal.h"

namespace htmsp {

namespace {

using namespace dev;

constexpr uint32_t kPerThread = kTileSynapses / kManyThreads;  // 16

// The instance descriptors live in device memory, so the compiler cannot
// tell that their pointers address global memory and would use flat
// accesses, which wait on LDS traffic too and do not batch; every access
// below goes through these global-space views instead.
#define HTMSP_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ HTMSP_G T* gbl(T* p) {
  return (HTMSP_G T*)p;
}

// A descriptor copied word by word through a global-space view.
template <typename T>
__device__ __forceinline__ T load_desc(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor size");
  T v;
  const HTMSP_G uint32_t* src = gbl(reinterpret_cast<const uint32_t*>(p));
  uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (uint32_t i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
  return v;
}

__device__ __forceinline__ uint64_t load_word(const HTMSP_G uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_word64(HTMSP_G uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_entry(const HTMSP_G uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_entry(HTMSP_G uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// floor(p / S) for p, S < 2^13 as one high multiply by m = ceil(2^32 / S)
// (exact there: the rounding error of m, times p, stays below 2^-6); S = 1,
// where m would not fit, is m = 0.
__device__ __forceinline__ uint32_t div_s(uint32_t p, uint32_t m) {
  return m ? __umulhi(p, m) : p;
}

struct TileLds {
  uint32_t cnt[kTileColumns];                 // raw overlap counts of the step
  uint16_t prev[kMaxTileSlots][kTileColumns];  // each tile's published overlaps of the last step
};
// a top-k workgroup reuses it for its waves' winner bitmaps
static_assert(sizeof(TileLds) >= 4 * 2 * kManyNV * 8 * sizeof(uint32_t), "top-k bitmaps");

// Step t of tile task `slot` of this workgroup, whole workgroup, once the
// scheduler has seen the instance's decision of step t - 1 (T, last tied
// winner + 1).  ALIGNED (S a multiple of 64): every 64-synapse chunk of a
// wave lies in one column, so the column, its "won" flag and its count are
// wave-uniform.
template <bool ALIGNED>
__device__ void tile_step(const ManyArgs& a, const ManyInst& in, uint32_t c0, uint32_t c1,
                          uint32_t t, uint32_t slot, TileLds& L, uint32_t T, uint32_t clast1) {
  const Shape& sh = in.sh;
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const uint32_t tag = (in.step_base + t + 1) & 0xFFFFu;
  const uint32_t ncol = c1 - c0, nsyn = ncol * sh.S;
  const bool learn_now = a.learn && t > 0;
  const bool overlap_now = t < in.F;
  const uint32_t m = in.smagic;

  const size_t p0 = (size_t)c0 * sh.S;
  HTMSP_G float* gperm = gbl(in.perm + p0);
  HTMSP_G uint32_t* gmir = gbl(in.mir + p0);
  // One packed word per synapse (index << 9 | q, from the launch's packing
  // pass); loads without branches (past the tile: its last synapse, then
  // ignored), so that all of them are in flight together.
  uint32_t ix[kPerThread], q[kPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kPerThread; ++j) ix[j] = gmir[min(tid + kManyThreads * j, nsyn - 1)];
#pragma unroll
  for (uint32_t j = 0; j < kPerThread; ++j) {
    const bool v = tid + kManyThreads * j < nsyn;
    q[j] = v ? ix[j] & 511u : 0u;
    ix[j] = v ? ix[j] >> 9 : 0u;
  }
  // column cl of this tile won frame t - 1 (its overlap of that frame is the
  // one this tile published last step)
  auto won_col = [&](uint32_t cl) {
    const uint32_t prev = L.prev[slot][cl];
    return prev > T || (T != 0 && prev == T && c0 + cl + 1 <= clast1);
  };

  // Both input gathers in one round: frame t - 1 for learning, frame t for
  // every synapse that can be connected after learning.
  const HTMSP_G uint32_t* fprev = gbl(in.frames + (size_t)(learn_now ? t - 1 : 0) * sh.W);
  const HTMSP_G uint32_t* fcur = gbl(in.frames + (size_t)(overlap_now ? t : 0) * sh.W);
  uint32_t won = 0;  // bit j: synapse j belongs to a winner
  uint32_t wp[kPerThread], wc[kPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kPerThread; ++j) {
    const uint32_t p = tid + kManyThreads * j;
    bool wj = false;
    if constexpr (ALIGNED) {
      const uint32_t pb = kManyThreads * j + kWave * wave;  // uniform
      wj = learn_now && pb < nsyn && won_col(div_s(pb, m));
    } else {
      wj = learn_now && p < nsyn && won_col(div_s(p, m));
    }
    won |= (uint32_t)wj << j;
    // unneeded gathers read word 0 (one cached line) instead of branching
    wp[j] = fprev[wj ? ix[j] >> 5 : 0u];
    const bool maybe = overlap_now && p < nsyn && (wj ? q[j] + sh.inc : q[j]) >= sh.theta;
    wc[j] = fcur[maybe ? ix[j] >> 5 : 0u];
  }
  if (won) {
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
      if (won & (1u << j)) {
        q[j] = learn_q(q[j], input_bit(wp[j], ix[j]), sh);
        gperm[tid + kManyThreads * j] = q_to_perm(q[j]);
        gmir[tid + kManyThreads * j] = (ix[j] << 9) | q[j];
      }
    }
  }
  if (overlap_now) {
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
      const uint32_t pb = kManyThreads * j + kWave * wave;  // first flat position of the chunk
      const bool hit = (pb + lane < nsyn) && q[j] >= sh.theta && input_bit(wc[j], ix[j]);
      const uint64_t mask = __ballot(hit);
      if (pb < nsyn && mask) {
        if constexpr (ALIGNED) {
          if (lane == 0) atomicAdd(&L.cnt[div_s(pb, m)], (uint32_t)__popcll(mask));
        } else {
          // columns that meet the chunk [pb, pb + 64): lane l counts column clA + l
          const uint32_t clA = div_s(pb, m);
          const uint32_t clB = div_s(min(pb + kWave, nsyn) - 1, m);
          const uint32_t cl = clA + lane;
          if (cl <= clB) {
            const uint32_t lo = max(cl * sh.S, pb) - pb;
            const uint32_t hi = min((cl + 1) * sh.S, pb + kWave) - pb;
            const uint64_t bits =
                hi - lo == 64 ? mask : (mask >> lo) & ((1ull << (hi - lo)) - 1);
            const uint32_t n = (uint32_t)__popcll(bits);
            if (n) atomicAdd(&L.cnt[cl], n);
          }
        }
      }
    }
  }
  __syncthreads();
  if (overlap_now) {
    for (uint32_t cl = tid; cl < ncol; cl += kManyThreads) {
      const uint32_t raw = L.cnt[cl];
      L.cnt[cl] = 0;
      const uint32_t ov = raw >= sh.m ? raw : 0u;
      L.prev[slot][cl] = (uint16_t)ov;
      store_entry(gbl(in.ovx) + c0 + cl, (tag << 16) | ov);
    }
  }
}

// Top-k task, one wave: collects the instance's overlaps of step t, resolves
// the global top-k, writes the outputs and publishes the decision.  Lane l
// holds columns u * 256 + 4l + q (q < 4) as the 16-bit fields of ev[u].
// Registers are kept to ev[] plus per-word temporaries past the first
// collection pass; the winners are ranked through bitmaps in the wave's LDS
// `bm` (2 kManyNV * 8 words).  Kept out of line: inlined, the compiler
// schedules its threshold search for registers that the tile path then
// pays for in occupancy.
// Returns false, having changed nothing, while some overlap of step t is
// not yet published.
__device__ __attribute__((noinline)) bool topk_try(ManyInst& in, uint32_t t, uint32_t lane,
                                                   uint32_t* bm) {
  const Shape& sh = in.sh;
  const uint32_t tag = (in.step_base + t + 1) & 0xFFFFu;
  // a stalled instance (failure-path tests) waits for a tag no tile writes
  const uint32_t want = in.stall ? (tag + 2) & 0xFFFFu : tag;
  const uint32_t nv = (sh.C + 4 * kWave - 1) / (4 * kWave);
  const HTMSP_G uint64_t* src = gbl(reinterpret_cast<const uint64_t*>(in.ovx));
  uint64_t ev[kManyNV];
#pragma unroll
  for (uint32_t u = 0; u < kManyNV; ++u) ev[u] = 0;
  // pair i holds columns c, c + 1 (c = (i / 2) * 256 + 4l + 2 (i % 2)); all
  // loads of a half are in flight at once.
  auto pair_col = [&](uint32_t i) { return (i / 2) * 4 * kWave + 4 * lane + 2 * (i % 2); };
  auto fresh = [&](uint64_t r, uint32_t c) {
    return (uint32_t)(r >> 16) % 65536u == want && (c + 1 >= sh.C || (uint32_t)(r >> 48) == want);
  };
  auto fold = [&](uint64_t r, uint32_t i, uint32_t c) {
    const uint64_t v = (r & 0xFFFFull) | (c + 1 < sh.C ? ((r >> 32) & 0xFFFFull) << 16 : 0ull);
    ev[i / 2] |= v << (32 * (i % 2));
  };
  uint32_t stale = 0;
  // (in two halves: 16 loads in flight, 1024 + 1024 columns, keep the
  // register peak of this pass below that of the tile path)
#pragma unroll
  for (uint32_t h = 0; h < 2; ++h) {
    if (h * kManyNV / 2 < nv) {
      uint64_t raw[kManyNV];
#pragma unroll
      for (uint32_t j = 0; j < kManyNV; ++j) {
        const uint32_t i = h * kManyNV + j, c = pair_col(i);
        raw[j] = (i / 2 < nv && c < sh.C) ? load_word(src + c / 2) : 0ull;
      }
#pragma unroll
      for (uint32_t j = 0; j < kManyNV; ++j) {
        const uint32_t i = h * kManyNV + j, c = pair_col(i);
        if (i / 2 < nv && c < sh.C) {
          if (fresh(raw[j], c)) fold(raw[j], i, c);
          else stale |= 1u << i;
        }
      }
    }
  }
  if (__any(stale != 0)) return false;
  uint32_t c_hi;
  const uint32_t T = topk_threshold(ev, sh.S, sh.k, in.guess, &c_hi);
  const uint32_t need = T ? sh.k - c_hi : 0u;
  const uint32_t nsel = T ? sh.k : c_hi;
  if (T) in.guess = T;

  // Winners in column order: every field above T, and the first `need`
  // fields equal to T.  The two field sets go into bitmaps of C bits in this
  // wave's LDS (bm: gt then eq, 128 words each); lane l then owns columns
  // 64 l .. 64 l + 63 (two words of each), takes its share of the ties and
  // writes its winners at their rank, two prefix counts over the lanes.
  HTMSP_G int32_t* wrow = gbl(in.win_out + (size_t)t * sh.k);
  HTMSP_G int32_t* ovrow = in.ov_out ? gbl(in.ov_out + (size_t)t * sh.C) : nullptr;
  HTMSP_G uint32_t* hist = in.hist ? gbl(in.hist) : nullptr;
  uint32_t* gtm = bm;
  uint32_t* eqm = bm + kManyNV * 8;
  for (uint32_t i = lane; i < kManyNV * 8; i += kWave) {
    gtm[i] = 0;
    eqm[i] = 0;
  }
  // the four field flags (bits 15, 31, 47, 63) of a word as a nibble
  auto nibble = [](uint64_t m) {
    return (uint32_t)(((m >> 15) & 1u) | ((m >> 30) & 2u) | ((m >> 45) & 4u) | ((m >> 60) & 8u));
  };
#pragma unroll
  for (uint32_t u = 0; u < kManyNV; ++u) {
    if (u < nv) {
      const uint64_t gt = field_add(ev[u], 0x7FFFu - T) & kHighBits;
      const uint64_t eq = T ? ((field_add(ev[u], 0x8000u - T) & kHighBits) & ~gt) : 0ull;
      // columns u * 256 + 4 l + q: word 8 u + l / 8, bits 4 (l mod 8) + q
      const uint32_t w = u * 8 + lane / 8, sft = 4 * (lane % 8);
      const uint32_t ng = nibble(gt), ne = nibble(eq);
      if (ng) atomicOr(&gtm[w], ng << sft);
      if (ne) atomicOr(&eqm[w], ne << sft);
      if (ovrow) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
          const uint32_t c = u * 4 * kWave + 4 * lane + q;
          if (c < sh.C) ovrow[c] = (int32_t)((ev[u] >> (16 * q)) & 0xFFFFu);
        }
      }
    }
  }
  const uint64_t gmask = (uint64_t)gtm[2 * lane] | ((uint64_t)gtm[2 * lane + 1] << 32);
  uint64_t emask = (uint64_t)eqm[2 * lane] | ((uint64_t)eqm[2 * lane + 1] << 32);
  const uint32_t neq = (uint32_t)__popcll(emask);
  const uint32_t eq_pre = wave_prefix<7>(neq, lane);
  uint32_t keep = need > eq_pre ? min(need - eq_pre, neq) : 0u;
  uint64_t take = 0;
  for (; keep > 0; --keep) {
    const uint64_t low = emask & (~emask + 1ull);
    take |= low;
    emask ^= low;
  }
  uint32_t clast1 = take ? 64 * lane + 64 - (uint32_t)__clzll((long long)take) : 0u;
  uint64_t sel = gmask | take;
  uint32_t pos = wave_prefix<7>((uint32_t)__popcll(sel), lane);
  while (sel) {
    const uint32_t c = 64 * lane + (uint32_t)__ffsll((long long)sel) - 1;
    wrow[pos++] = (int32_t)c;
    // this wave is the instance's only histogram writer in the launch
    if (hist) hist[c] += 1u;
    sel &= sel - 1ull;
  }
  for (uint32_t i = nsel + lane; i < sh.k; i += kWave) wrow[i] = -1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) clast1 = max(clast1, (uint32_t)__shfl_xor(clast1, off));
  if (lane == 0)
    store_word64(gbl(in.dec), ((uint64_t)tag << 48) | ((uint64_t)T << 32) | (uint64_t)clast1);
  return true;
}

// Two waves per SIMD (at most 256 registers): two tiles in flight per CU
// already keep more bytes in flight than device memory needs to stream.
// ALIGNED: every instance of the launch has S a multiple of 64 (one tile
// path per kernel keeps the register allocation free of spills).
//
// A workgroup holds either tile tasks only or top-k tasks only.  A tile
// workgroup runs whichever of its tiles can take its next step (the
// instance's decision of the tile's previous step is out), so a tile whose
// instance is late never holds up the others; thread 0 finds the tile and
// the whole workgroup runs its step.  In a top-k workgroup every wave polls
// its own instances (tasks j with j % 4 == wave) and resolves any whose
// overlaps of its next step are all published.  Both loops end when every
// task has taken all its steps, or on abort (spin limit or the launch's error
// word); a workgroup that gives up also sets the error word of every instance
// it holds a task of, so that each affected handle reports the failure.
template <bool ALIGNED>
__global__ __launch_bounds__(kManyThreads, 2) void k_sp_many(ManyArgs a) {
  constexpr uint32_t kSlots = kMaxTopkSlots > kMaxTileSlots ? kMaxTopkSlots : kMaxTileSlots;
  __shared__ TileLds L;
  // this workgroup's tasks and their instances, read from device memory once
  __shared__ ManyTask s_task[kSlots];
  __shared__ ManyInst s_inst[kSlots];
  __shared__ uint32_t s_next[kSlots];  // each task's next step
  __shared__ uint32_t s_pick[4];      // chosen tile, T, last tied winner + 1, status
  const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  for (uint32_t i = tid; i < kTileColumns; i += kManyThreads) L.cnt[i] = 0;
  const HTMSP_G uint32_t* task_off = gbl(a.task_off);
  const uint32_t t0 = task_off[blockIdx.x], t1 = task_off[blockIdx.x + 1];
  const uint32_t nt = min(t1 - t0, kSlots);
  for (uint32_t i = tid; i < nt; i += kManyThreads) {
    s_task[i] = load_desc(a.tasks + t0 + i);
    s_inst[i] = load_desc(a.insts + s_task[i].inst);
    s_next[i] = 0;
  }
  __syncthreads();
  if (nt == 0) return;  // whole workgroup
  HTMSP_G uint32_t* err = gbl(a.err);

  if (s_task[0].kind == 1) {
    // ---- top-k workgroup: each wave on its own instances, no barriers ----
    bool fail = t1 - t0 > kMaxTopkSlots;
    uint32_t spins = 0;
    while (!fail) {
      bool all_done = true, progress = false;
      for (uint32_t j = wave; j < nt; j += kManyThreads / kWave) {
        const uint32_t t = s_next[j];
        if (t >= s_inst[j].F) continue;
        all_done = false;
        if (topk_try(s_inst[j], t, lane, reinterpret_cast<uint32_t*>(&L) + wave * kManyNV * 16)) {
          s_next[j] = t + 1;  // every lane: each keeps its own view of the slot exact
          progress = true;
        }
      }
      if (all_done) break;
      if (progress) {
        spins = 0;
      } else {
        if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_entry(err) != 0)) fail = true;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (fail && lane == 0) {
      store_entry(err, 1u);
      // this wave's instances may be part-way through a step
      for (uint32_t j = wave; j < nt; j += kManyThreads / kWave) store_entry(gbl(s_inst[j].err), 1u);
    }
    return;
  }

  // ---- tile workgroup ----
  // The launch's packed copy of each tile's synapses, written by the thread
  // that reads it in every step (same flat positions), so each step loads
  // one word per synapse instead of an index and a permanence.
  for (uint32_t j = 0; j < nt && t1 - t0 <= kMaxTileSlots; ++j) {
    const ManyInst& in = s_inst[j];
    const size_t p0 = (size_t)s_task[j].c0 * in.sh.S;
    const uint32_t nsyn = (s_task[j].c1 - s_task[j].c0) * in.sh.S;
    const HTMSP_G uint32_t* gidx = gbl(in.idx + p0);
    const HTMSP_G float* gperm = gbl(in.perm + p0);
    HTMSP_G uint32_t* gmir = gbl(in.mir + p0);
    for (uint32_t p = tid; p < nsyn; p += kManyThreads)
      gmir[p] = (min(gidx[p], in.sh.N - 1) << 9) | perm_to_q(gperm[p]);
  }
  // Wave 0 looks at every tile at once (lane j: tile j) and takes the first
  // ready one at or after `rr`, so that no tile is passed over for long.
  // The decision words it looks at were loaded while the previous tile step
  // ran (issued with that step's state loads, so the two latencies overlap);
  // a word loaded before its decision was published only makes a tile look
  // not ready yet (readiness is an exact tag match), and when no tile looks
  // ready the words are loaded again.
  uint32_t rr = 0, spins = 0;
  uint64_t dpre = 0;
  bool have = false;
  while (true) {
    if (wave == 0) {
      uint32_t status = 3, pick = 0, T = 0, clast1 = 0;  // 3: nothing ready yet
      if (t1 - t0 > kMaxTileSlots) {
        status = 2;
      } else {
        const uint32_t j = lane < nt ? lane : 0u;
        const uint32_t t = s_next[j];
        const bool live = lane < nt && t <= s_inst[j].F;
        uint64_t d = dpre;
        if (!have) d = (live && t > 0) ? load_word(gbl(s_inst[j].dec)) : 0ull;
        have = false;
        const bool ready =
            live && (t == 0 || (uint32_t)(d >> 48) == ((s_inst[j].step_base + t) & 0xFFFFu));
        const uint64_t lm = __ballot(live), rm = __ballot(ready);
        if (lm == 0) {
          status = 1;
        } else if (rm == 0) {
          if (++spins > a.spin_limit || ((spins & 63u) == 0 && load_entry(err) != 0))
            status = 2;
          else
            __builtin_amdgcn_s_sleep(1);
        } else {
          const uint64_t after = rm & (~0ull << rr);
          pick = (uint32_t)__ffsll((long long)(after ? after : rm)) - 1;
          T = (uint32_t)__shfl((int)((uint32_t)(d >> 32) & 0xFFFFu), (int)pick);
          clast1 = (uint32_t)__shfl((int)(uint32_t)d, (int)pick);
          status = 0;
          spins = 0;
          rr = pick + 1;  // at most kMaxTileSlots < 64
        }
      }
      if (lane == 0) {
        s_pick[0] = pick;
        s_pick[1] = T;
        s_pick[2] = clast1;
        s_pick[3] = status;
      }
    }
    __syncthreads();
    const uint32_t status = s_pick[3];
    if (status == 1) break;
    if (status == 2) {
      if (tid == 0) {
        store_entry(err, 1u);
        // the instances of this workgroup's tiles may be part-way through a step
        for (uint32_t j = 0; j < nt; ++j) store_entry(gbl(s_inst[j].err), 1u);
      }
      break;
    }
    if (status == 0) {
      const uint32_t j = s_pick[0];
      const ManyTask& task = s_task[j];
      if (wave == 0) {
        // the decisions the next pick looks at (the picked tile's own word is
        // still that of its current step, so it looks not ready, as it is)
        const uint32_t jj = lane < nt ? lane : 0u;
        const uint32_t tt = s_next[jj];
        dpre = (lane < nt && tt > 0 && tt <= s_inst[jj].F) ? load_word(gbl(s_inst[jj].dec))
                                                            : 0ull;
        have = true;
      }
      tile_step<ALIGNED>(a, s_inst[j], task.c0, task.c1, s_next[j], j, L, s_pick[1], s_pick[2]);
      // every thread has read s_next[j] and s_pick before tile_step's barrier
      if (tid == 0) s_next[j] += 1;
    }
    __syncthreads();
  }
}

}  // namespace

uint32_t many_tile_columns(uint32_t S) {
  return std::min(kTileColumns, std::max(1u, kTileSynapses / S));
}

static const void* many_kernel(bool aligned) {
  return aligned ? reinterpret_cast<const void*>(&k_sp_many<true>)
                 : reinterpret_cast<const void*>(&k_sp_many<false>);
}

hipError_t launch_many(const ManyArgs& a, uint32_t grid, bool aligned, hipStream_t s) {
  ManyArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(many_kernel(aligned), dim3(grid), dim3(kManyThreads), args,
                                    0, s);
}

int many_max_blocks(int device, bool aligned) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, many_kernel(aligned), kManyThreads,
                                                   0) != hipSuccess)
    return 0;
  return cus * per_cu;
}

}  // namespace htmsp
